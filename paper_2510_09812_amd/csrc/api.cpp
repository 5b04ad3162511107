// C ABI of the GSPM library: argument checking, state machine, host<->device
// marshalling in the caller's node order.  Every numerical step runs in the
// HIP kernels; this file only moves data and sequences calls.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "context.h"

using namespace gspm;

namespace {

thread_local std::string g_create_error = "no error";

constexpr int kRing = 520;        // CG dot-product slots: >= largest iteration batch + 2

gspm_status fail(gspm_ctx *c, gspm_status s, const std::string &msg) {
    if (c) c->err = msg;
    return s;
}

// Device buffers of a mesh upload come from one arena (one hipMalloc, each
// buffer 256-byte aligned): one large allocation is placed in large
// contiguous fragments, where separate ones can land fragmented among other
// allocations of the process and run the gathers of the element kernels
// measurably slower.  In planning mode dev_alloc only adds up the sizes;
// outside the arena (or past its end) it falls back to hipMalloc.
constexpr size_t kArenaAlign = 256;

}  // namespace

namespace gspm {

int ctx_malloc(gspm_ctx *c, void **p, size_t bytes, const char *what) {
    *p = nullptr;
    if (c->alloc_fn) {
        *p = c->alloc_fn(bytes, c->alloc_user);
        if (!*p) {
            c->err = std::string(what) + ": the caller's allocator returned NULL";
            return GSPM_E_OOM;
        }
        return GSPM_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return hip_check(c, e, what);
    }
    return GSPM_OK;
}

void ctx_free(const gspm_ctx *c, void *p) {
    if (!p) return;
    if (c->free_fn) c->free_fn(p, c->alloc_user);
    else hipFree(p);
}

}  // namespace gspm

namespace {

template <class T>
int dev_alloc(gspm_ctx *c, T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    const size_t bytes = (sizeof(T) * count + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
    if (c->arena_planning) {
        c->arena_size += bytes;
        return GSPM_OK;
    }
    if (c->arena && c->arena_used + bytes <= c->arena_size) {
        *p = reinterpret_cast<T *>(c->arena + c->arena_used);
        c->arena_used += bytes;
        return GSPM_OK;
    }
    void *v = nullptr;
    const int rc = ctx_malloc(c, &v, sizeof(T) * count, "device allocation");
    *p = static_cast<T *>(v);
    return rc;
}

template <class T>
void dev_free(const gspm_ctx *c, T *&p) {
    const char *q = reinterpret_cast<const char *>(p);
    if (p && !(c->arena && q >= c->arena && q < c->arena + c->arena_size)) ctx_free(c, const_cast<void *>(static_cast<const void *>(p)));
    p = nullptr;
}

bool all_finite(const double *v, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

int upload(gspm_ctx *c, double *dst, const std::vector<double> &h) {
    int rc = hip_check(c, hipMemcpyAsync(dst, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, c->stream),
                       "copy to device");
    if (rc) return rc;
    return hip_check(c, hipStreamSynchronize(c->stream), "copy to device");
}

int download(gspm_ctx *c, const double *src, std::vector<double> &h) {
    int rc = hip_check(c, hipMemcpyAsync(h.data(), src, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->stream),
                       "copy to host");
    if (rc) return rc;
    return hip_check(c, hipStreamSynchronize(c->stream), "copy to host");
}

// Homogeneous strain of an applied stress for cubic C:
// normal part eps = (sigma - c12 tr(sigma) / (c11 + 2 c12)) / (c11 - c12),
// shear eps_ij = sigma_ij / (2 c44).
void cubic_compliance(const gspm_params &p, const double s[6], double e[6]) {
    const double tr = s[0] + s[1] + s[2];
    for (int k = 0; k < 3; ++k) e[k] = (s[k] - p.c12 * tr / (p.c11 + 2.0 * p.c12)) / (p.c11 - p.c12);
    for (int k = 3; k < 6; ++k) e[k] = s[k] / (2.0 * p.c44);
}

// A symmetric tensor (xx yy zz yz xz xy): R A R^T or R^T A R.
void rotate_sym(const double R[9], bool to_sample, const double a[6], double b[6]) {
    const double A[3][3] = {{a[0], a[5], a[4]}, {a[5], a[1], a[3]}, {a[4], a[3], a[2]}};
    double Q[3][3], B[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Q[i][j] = to_sample ? R[3 * i + j] : R[3 * j + i];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double v = 0.0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) v += Q[i][k] * A[k][l] * Q[j][l];
            B[i][j] = v;
        }
    b[0] = B[0][0]; b[1] = B[1][1]; b[2] = B[2][2]; b[3] = B[1][2]; b[4] = B[0][2]; b[5] = B[0][1];
}

// The cubic stiffness seen from the sample frame (App. D) as a Voigt matrix
// (xx yy zz yz xz xy, engineering shear): the Bond transformation M C M^T,
// with M the stress-type rotation of Voigt vectors built from R.
void sample_stiffness(const gspm_params &p, const double R[9], double C6[36]) {
    static const int ij[6][2] = {{0, 0}, {1, 1}, {2, 2}, {1, 2}, {0, 2}, {0, 1}};
    double C[6][6] = {}, M[6][6];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) C[i][j] = p.c12;
        C[i][i] = p.c11;
        C[3 + i][3 + i] = p.c44;
    }
    // row r of M: sigma'_r = sum_c M_rc sigma_c for sigma' = R sigma R^T
    for (int r = 0; r < 6; ++r) {
        const int a = ij[r][0], b = ij[r][1];
        for (int col = 0; col < 6; ++col) {
            const int k = ij[col][0], l = ij[col][1];
            M[r][col] = k == l ? R[3 * a + k] * R[3 * b + k] : R[3 * a + k] * R[3 * b + l] + R[3 * a + l] * R[3 * b + k];
        }
    }
    for (int r = 0; r < 6; ++r)
        for (int col = 0; col < 6; ++col) {
            double v = 0.0;
            for (int x = 0; x < 6; ++x)
                for (int y = 0; y < 6; ++y) v += M[r][x] * C[x][y] * M[col][y];
            C6[6 * r + col] = v;
        }
}

}  // namespace

namespace gspm {

// Caller-order n0 x 3 -> internal component-major 3 x n.  The copies of a
// periodic node must agree to 1e-12 relative.
int gather_user(gspm_ctx *c, const double *v, std::vector<double> &out) {
    const int n = c->n;
    out.assign(3 * static_cast<size_t>(n), 0.0);
    std::vector<uint8_t> seen(static_cast<size_t>(n), 0);
    for (int64_t i = 0; i < c->n0; ++i) {
        const int32_t k = c->user2int[i];
        for (int a = 0; a < 3; ++a) {
            const double x = v[i * 3 + a];
            if (!std::isfinite(x)) {
                c->err = "non-finite value in a nodal field";
                return GSPM_E_ARG;
            }
            double &dst = out[static_cast<size_t>(a) * n + k];
            if (!seen[k]) dst = x;
            else if (std::fabs(dst - x) > 1e-12 * std::max(std::fabs(dst), std::fabs(x))) {
                c->err = "periodic copies of a node carry different values";
                return GSPM_E_ARG;
            }
        }
        seen[k] = 1;
    }
    return GSPM_OK;
}

void scatter_user(const gspm_ctx *c, const std::vector<double> &in, double *out) {
    const int n = c->n;
    for (int64_t i = 0; i < c->n0; ++i) {
        const int32_t k = c->user2int[i];
        for (int a = 0; a < 3; ++a) out[i * 3 + a] = in[static_cast<size_t>(a) * n + k];
    }
}

}  // namespace gspm

gspm_ctx::~gspm_ctx() {
    release_nn();
    release_mesh();
    release_pc();
    for (auto &pl : prof)
        for (hipEvent_t e : pl.ev) hipEventDestroy(e);
    for (hipEvent_t e : ev)
        if (e) hipEventDestroy(e);
    if (t0) hipEventDestroy(t0);
    if (t1) hipEventDestroy(t1);
    for (hipEvent_t e : phase_ev)
        if (e) hipEventDestroy(e);
    if (h_flags) hipHostFree(h_flags);
    if (h_mixed) hipHostFree(h_mixed);
    if (h_step) hipHostFree(h_step);
    if (own_stream && stream) hipStreamDestroy(stream);
}

void gspm_ctx::release_mesh() {
    if (stream) hipStreamSynchronize(stream);
    release_pc();
    auto &b = d;
    dev_free(this, b.x); dev_free(this, b.lconn); dev_free(this, b.blk_ptr); dev_free(this, b.blk_nmag); dev_free(this, b.w);
    dev_free(this, b.halo_ptr); dev_free(this, b.halo_ids); dev_free(this, b.halo_lo); dev_free(this, b.img);
    dev_free(this, b.stc64); dev_free(this, b.stc32); dev_free(this, b.seg_ent); dev_free(this, b.seg_off); dev_free(this, b.seg_nel); dev_free(this, b.seg_ptr); dev_free(this, b.seg_nmag);
    dev_free(this, b.m); dev_free(this, b.mnext); dev_free(this, b.u); dev_free(this, b.unext);
    dev_free(this, b.ms); dev_free(this, b.g); dev_free(this, b.gs); dev_free(this, b.b); dev_free(this, b.ch2);
    dev_free(this, b.r); dev_free(this, b.p); dev_free(this, b.p2); dev_free(this, b.q); dev_free(this, b.r2); dev_free(this, b.q2);
    dev_free(this, b.sums); dev_free(this, b.esums); dev_free(this, b.dm); dev_free(this, b.der); dev_free(this, b.bad);
    dev_free(this, b.cg_rr); dev_free(this, b.cg_pq); dev_free(this, b.cg_bb); dev_free(this, b.cg_rq); dev_free(this, b.cg_qq); dev_free(this, b.cg_flags);
    dev_free(this, b.r32); dev_free(this, b.p32); dev_free(this, b.p32b); dev_free(this, b.q32); dev_free(this, b.x32); dev_free(this, b.r32b);
    dev_free(this, b.q32b);
    dev_free(this, b.cgi_rr); dev_free(this, b.cgi_pq); dev_free(this, b.cgi_bb); dev_free(this, b.cgi_rq); dev_free(this, b.cgi_qq);
    dev_free(this, b.cgi_flags);
    dev_free(this, b.gcorr); dev_free(this, b.gstart);
    dev_free(this, b.mprev); dev_free(this, b.uprev); dev_free(this, b.du_prev); dev_free(this, b.kdu); dev_free(this, b.wred); dev_free(this, b.wcoef);
    dev_free(this, b.ud); dev_free(this, b.udnext); dev_free(this, b.rep);
    dev_free(this, b.cg_rz); dev_free(this, b.cgi_rz);
    dev_free(this, b.cg_rzq); dev_free(this, b.cg_qzq); dev_free(this, b.cgi_rzq); dev_free(this, b.cgi_qzq);
    dev_free(this, b.det_part); dev_free(this, b.det_dst); dev_free(this, b.det_count); dev_free(this, b.inc_ptr);
    dev_free(this, b.inc_ent);
    dev_free(this, b.gs_halo_ptr); dev_free(this, b.gs_halo_ids);
    dev_free(this, b.gs_off); dev_free(this, b.gs_col); dev_free(this, b.gs_kv); dev_free(this, b.gs_mv);
    dev_free(this, b.gs_kd); dev_free(this, b.gs_md);
    for (int k = 0; k < 2; ++k) {
        dev_free(this, b.gs_a64[k]); dev_free(this, b.gs_d64[k]); dev_free(this, b.gs_a32[k]); dev_free(this, b.gs_d32[k]);
        gs_slot[k] = gspm::GsSlot{};
    }
    gs_nent = 0;
    if (arena) gspm::ctx_free(this, arena);
    arena = nullptr;
    arena_size = arena_used = 0;
    have_mesh = have_m = have_prev = false;
    gcorr_ok = 0;
    commits = 0;
    tets_int.clear();
    release_nn();
}

void gspm_ctx::release_nn() {
    if (stream) hipStreamSynchronize(stream);
    auto &q = nn;
    dev_free(this, q.gptr); dev_free(this, q.gnbr); dev_free(this, q.master); dev_free(this, q.wr); dev_free(this, q.m1); dev_free(this, q.m2);
    dev_free(this, q.grad); dev_free(this, q.mats); dev_free(this, q.acts); dev_free(this, q.y); dev_free(this, q.red); dev_free(this, q.dvec);
    dev_free(this, q.du); dev_free(this, q.mp_in); dev_free(this, q.m_in);
    dev_free(this, q.gh); dev_free(this, q.gha); dev_free(this, q.gab); dev_free(this, q.gy); dev_free(this, q.part);
    q = gspm::MpnnState{};
    warm_mode = GSPM_WARM_PREVIOUS;
}

extern "C" {

gspm_status gspm_create(gspm_ctx **out, const gspm_create_opts *opts) {
    if (!out) {
        g_create_error = "gspm_create: null output pointer";
        return GSPM_E_ARG;
    }
    *out = nullptr;
    gspm_create_opts o{};
    if (opts) o = *opts;
    if (o.precision != GSPM_FP64 && o.precision != GSPM_MIXED) {
        g_create_error = "gspm_create: unknown precision";
        return GSPM_E_ARG;
    }
    if (o.reorder != GSPM_REORDER_MORTON && o.reorder != GSPM_REORDER_NONE && o.reorder != GSPM_REORDER_RCM) {
        g_create_error = "gspm_create: unknown reorder";
        return GSPM_E_ARG;
    }
    if ((o.dev_alloc == nullptr) != (o.dev_free == nullptr)) {
        g_create_error = "gspm_create: dev_alloc and dev_free go together";
        return GSPM_E_ARG;
    }
    if (o.block_nodes != 0 && (o.block_nodes < 64 || o.block_nodes > 1024 || (o.block_nodes & (o.block_nodes - 1)))) {
        g_create_error = "gspm_create: block_nodes must be 0 or a power of two in [64, 1024]";
        return GSPM_E_ARG;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        g_create_error = "gspm_create: no HIP device available";
        return GSPM_E_DEVICE;
    }
    if (o.device < 0 || o.device >= ndev) {
        g_create_error = "gspm_create: device ordinal out of range";
        return GSPM_E_ARG;
    }
    hipDeviceProp_t prop;
    if (hipSetDevice(o.device) != hipSuccess || hipGetDeviceProperties(&prop, o.device) != hipSuccess) {
        g_create_error = "gspm_create: cannot use the device";
        return GSPM_E_DEVICE;
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        g_create_error = std::string("gspm_create: the library is built for gfx950, device is ") + prop.gcnArchName;
        return GSPM_E_DEVICE;
    }
    auto *c = new gspm_ctx();
    c->device = o.device;
    c->precision = o.precision;
    c->block_nodes = o.block_nodes;
    c->reorder = o.reorder;
    c->deterministic = o.deterministic != 0;
    c->alloc_fn = o.dev_alloc;
    c->free_fn = o.dev_free;
    c->alloc_user = o.alloc_user;
    c->profile = o.profile != 0;
    if (o.stream) {
        c->stream = static_cast<hipStream_t>(o.stream);
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            g_create_error = "gspm_create: cannot create a stream";
            return GSPM_E_DEVICE;
        }
        c->own_stream = true;
    }
    // coherent: kernels write the convergence flags and residual totals here directly
    bool ok = hipHostMalloc(reinterpret_cast<void **>(&c->h_flags), sizeof(int32_t) * 4 * kMaxComp,
                            hipHostMallocCoherent) == hipSuccess;
    ok = ok && hipHostMalloc(reinterpret_cast<void **>(&c->h_mixed), sizeof(double) * 16 * kShards,
                             hipHostMallocCoherent) == hipSuccess;
    ok = ok && hipHostMalloc(reinterpret_cast<void **>(&c->h_step), sizeof(double) * 16, hipHostMallocCoherent) ==
                   hipSuccess;
    for (auto &e : c->ev) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreate(&c->t0) == hipSuccess && hipEventCreate(&c->t1) == hipSuccess;
    for (auto &e : c->phase_ev) ok = ok && hipEventCreate(&e) == hipSuccess;
    if (!ok) {
        delete c;
        g_create_error = "gspm_create: cannot allocate host resources";
        return GSPM_E_DEVICE;
    }
    // the allocation-free entry point's scratch: its address on this device,
    // looked up once per device with the device current
    if (noalloc_scratch_address(o.device, &c->na_scratch) != 0 || !c->na_scratch) {
        delete c;
        g_create_error = "gspm_create: cannot look up the device address of the fixed scratch";
        return GSPM_E_DEVICE;
    }
    c->err = "no error";
    *out = c;
    return GSPM_OK;
}

void gspm_destroy(gspm_ctx *ctx) {
    if (!ctx) return;
    hipSetDevice(ctx->device);
    delete ctx;
}

gspm_status gspm_upload_mesh(gspm_ctx *c, int64_t n_nodes, const double *xyz, int64_t n_tets, const int32_t *tets,
                             const uint8_t *tags, const double lo[3], const double hi[3], uint32_t flags) {
    if (!c) return GSPM_E_ARG;
    if (!xyz || !tets || !tags || !lo || !hi) return fail(c, GSPM_E_ARG, "upload_mesh: null array");
    if (!(flags & GSPM_PERIODIC)) return fail(c, GSPM_E_ARG, "upload_mesh: only periodic cells are supported");
    hipSetDevice(c->device);
    HostMesh hm;
    std::string err;
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess)
        return fail(c, GSPM_E_DEVICE, "upload_mesh: cannot query the LDS size");
    int32_t nb = nodes_per_block(c->block_nodes, n_nodes);
    int rc;
    for (;;) {
        rc = prepare_mesh(n_nodes, xyz, n_tets, tets, tags, lo, hi, nb, hm, err, c->reorder);
        if (rc) return fail(c, static_cast<gspm_status>(rc), "upload_mesh: " + err);
        const size_t need = elem_lds_bytes(hm.nb, hm.nloc_max);
        if (need <= static_cast<size_t>(lds_max)) break;
        if (c->block_nodes != 0 || nb <= 64)
            return fail(c, GSPM_E_ARG, "upload_mesh: blocks of " + std::to_string(nb) + " nodes need " +
                                           std::to_string(need) + " bytes of LDS per workgroup, the device has " +
                                           std::to_string(lds_max) + "; use smaller block_nodes");
        nb /= 2;                   // automatic block size: halve until the element kernels fit
    }
    // GS row blocks: four times the element blocks (at most 1024 nodes) in
    // the mixed form, whose FP32 row kernels stage 16 bytes per node (two
    // workgroups per CU; the per-workgroup work of a CG iteration is spread
    // over more rows); the element blocks' size in FP64 contexts (FP64
    // staging would cut occupancy further)
    GsRowsHost rows;
    const bool fp64_cg = c->precision != GSPM_MIXED;
    const int32_t nb_rows = fp64_cg ? hm.nb : std::max(hm.nb, std::min(4 * hm.nb, 1024));
    rc = assemble_gs_rows(hm, n_tets, tets, tags, nb_rows, rows, err);
    if (!rc && rows.nb != hm.nb && rows_lds_bytes(rows.nb, rows.nloc_max, fp64_cg) > static_cast<size_t>(lds_max))
        rc = assemble_gs_rows(hm, n_tets, tets, tags, hm.nb, rows, err);
    if (rc) return fail(c, static_cast<gspm_status>(rc), "upload_mesh: " + err);
    if (rows_lds_bytes(rows.nb, rows.nloc_max, fp64_cg) > static_cast<size_t>(lds_max))
        return fail(c, GSPM_E_ARG, "upload_mesh: the GS row blocks need more LDS than the device has; use smaller "
                                   "block_nodes");
    // deterministic mode: per owned node its element copies, (copy index within the block's list) << 2 | slot
    std::vector<int32_t> inc_ptr;
    std::vector<uint16_t> inc_ent;
    int32_t det_blocks = 0;
    if (c->deterministic) {
        const size_t nslot = static_cast<size_t>(hm.nblk) * hm.nb;
        inc_ptr.assign(nslot + 1, 0);
        for (int32_t b = 0; b < hm.nblk; ++b) {
            if (hm.blk_ptr[b + 1] - hm.blk_ptr[b] > 16384)
                return fail(c, GSPM_E_ARG, "upload_mesh: deterministic mode needs at most 16384 element copies per "
                                           "block; use smaller block_nodes");
            for (int32_t e = hm.blk_ptr[b]; e < hm.blk_ptr[b + 1]; ++e)
                for (int j = 0; j < 4; ++j) {
                    const int v = hm.lconn[4 * static_cast<size_t>(e) + j];
                    if (v < hm.nb) ++inc_ptr[static_cast<size_t>(b) * hm.nb + v + 1];
                }
        }
        for (size_t i = 0; i < nslot; ++i) inc_ptr[i + 1] += inc_ptr[i];
        inc_ent.resize(static_cast<size_t>(inc_ptr[nslot]));
        std::vector<int32_t> cur(inc_ptr.begin(), inc_ptr.end() - 1);
        for (int32_t b = 0; b < hm.nblk; ++b)
            for (int32_t e = hm.blk_ptr[b]; e < hm.blk_ptr[b + 1]; ++e)
                for (int j = 0; j < 4; ++j) {
                    const int v = hm.lconn[4 * static_cast<size_t>(e) + j];
                    if (v < hm.nb)
                        inc_ent[static_cast<size_t>(cur[static_cast<size_t>(b) * hm.nb + v]++)] =
                            static_cast<uint16_t>(((e - hm.blk_ptr[b]) << 2) | j);
                }
        // the largest grid of a launch that adds sums: the element passes (one workgroup per block) and the
        // node passes (at most 2048, or one thread per node)
        det_blocks = std::max({2048, hm.nblk, (hm.n + kThreads - 1) / kThreads});
    }
    c->release_mesh();
    const size_t n = static_cast<size_t>(hm.n), n3 = 3 * n;
    const size_t nent = rows.col.size();
    auto &d = c->d;
    const size_t nstc = static_cast<size_t>(hm.nblk) * hm.nb + hm.halo_ids.size();
    const size_t nseg = hm.seg_nel.size();
    auto alloc_all = [&]() -> int {
        int rc = 0;
        rc = rc ? rc : dev_alloc(c, &d.x, n3);
        rc = rc ? rc : dev_alloc(c, &d.lconn, static_cast<size_t>(hm.ncopies));
        rc = rc ? rc : dev_alloc(c, &d.blk_ptr, hm.blk_ptr.size());
        rc = rc ? rc : dev_alloc(c, &d.blk_nmag, hm.blk_nmag.size());
        rc = rc ? rc : dev_alloc(c, &d.halo_ptr, hm.halo_ptr.size());
        rc = rc ? rc : dev_alloc(c, &d.halo_ids, hm.halo_ids.size());
        rc = rc ? rc : dev_alloc(c, &d.halo_lo, hm.halo_lo.size());
        rc = rc ? rc : dev_alloc(c, &d.img, hm.img.size());
        rc = rc ? rc : dev_alloc(c, &d.w, n);
        rc = rc ? rc : dev_alloc(c, &d.stc64, 3 * nstc);
        rc = rc ? rc : dev_alloc(c, &d.stc32, 3 * nstc);
        rc = rc ? rc : dev_alloc(c, &d.seg_ent, hm.seg_ent.size() / 8);
        rc = rc ? rc : dev_alloc(c, &d.seg_off, nseg);
        rc = rc ? rc : dev_alloc(c, &d.seg_nel, nseg);
        rc = rc ? rc : dev_alloc(c, &d.seg_ptr, hm.seg_ptr.size());
        rc = rc ? rc : dev_alloc(c, &d.seg_nmag, hm.seg_nmag.size());
        for (double **p : {&d.m, &d.mnext, &d.u, &d.unext, &d.ms, &d.g, &d.gs, &d.b, &d.r, &d.p, &d.p2, &d.q, &d.r2, &d.q2,
                            &d.mprev, &d.uprev, &d.du_prev, &d.kdu, &d.gstart})
            rc = rc ? rc : dev_alloc(c, p, n3);
        rc = rc ? rc : dev_alloc(c, &d.gcorr, 8 * static_cast<size_t>(n));
        rc = rc ? rc : dev_alloc(c, &d.ud, n);
        rc = rc ? rc : dev_alloc(c, &d.udnext, n);
        rc = rc ? rc : dev_alloc(c, &d.rep, n);
        rc = rc ? rc : dev_alloc(c, &d.cg_rz, static_cast<size_t>(kMaxComp) * kRing * kShards);
        rc = rc ? rc : dev_alloc(c, &d.cg_rzq, static_cast<size_t>(kMaxComp) * kRing * kShards);
        rc = rc ? rc : dev_alloc(c, &d.cg_qzq, static_cast<size_t>(kMaxComp) * kRing * kShards);
        rc = rc ? rc : dev_alloc(c, &d.gs_off, rows.off.size());
        rc = rc ? rc : dev_alloc(c, &d.gs_halo_ptr, rows.halo_ptr.size());
        if (!rows.halo_ids.empty()) rc = rc ? rc : dev_alloc(c, &d.gs_halo_ids, rows.halo_ids.size());
        rc = rc ? rc : dev_alloc(c, &d.gs_col, nent);
        rc = rc ? rc : dev_alloc(c, &d.gs_kv, nent);
        rc = rc ? rc : dev_alloc(c, &d.gs_mv, nent);
        rc = rc ? rc : dev_alloc(c, &d.gs_kd, n);
        rc = rc ? rc : dev_alloc(c, &d.gs_md, n);
        if (c->deterministic) {
            rc = rc ? rc : dev_alloc(c, &d.inc_ptr, inc_ptr.size());
            rc = rc ? rc : dev_alloc(c, &d.inc_ent, inc_ent.size());
            rc = rc ? rc : dev_alloc(c, &d.det_part, static_cast<size_t>(kDetSlots) * det_blocks);
            rc = rc ? rc : dev_alloc(c, &d.det_dst, static_cast<size_t>(kDetSlots));
            rc = rc ? rc : dev_alloc(c, &d.det_count, 1);
        }
        for (int k = 0; k < 2; ++k) {
            rc = rc ? rc : dev_alloc(c, &d.gs_a64[k], nent);
            rc = rc ? rc : dev_alloc(c, &d.gs_d64[k], n);
        }
        rc = rc ? rc : dev_alloc(c, &d.wred, static_cast<size_t>(mpnn::kMrSums) * kShards);
        rc = rc ? rc : dev_alloc(c, &d.wcoef, 2);
        rc = rc ? rc : dev_alloc(c, &d.ch2, 2 * n);
        rc = rc ? rc : dev_alloc(c, &d.sums, 9 * kShards);
        rc = rc ? rc : dev_alloc(c, &d.esums, 5 * kShards);
        rc = rc ? rc : dev_alloc(c, &d.dm, kShards);
        rc = rc ? rc : dev_alloc(c, &d.der, 2);
        rc = rc ? rc : dev_alloc(c, &d.bad, 1);
        rc = rc ? rc : dev_alloc(c, &d.cg_rr, static_cast<size_t>(kMaxComp) * kRing * kShards);
        rc = rc ? rc : dev_alloc(c, &d.cg_pq, static_cast<size_t>(kMaxComp) * kRing * kShards);
        rc = rc ? rc : dev_alloc(c, &d.cg_bb, static_cast<size_t>(kMaxComp) * kShards);
        rc = rc ? rc : dev_alloc(c, &d.cg_rq, static_cast<size_t>(kRing) * kShards);
        rc = rc ? rc : dev_alloc(c, &d.cg_qq, static_cast<size_t>(kRing) * kShards);
        rc = rc ? rc : dev_alloc(c, &d.cg_flags, 2 * kMaxComp);
        if (c->precision == GSPM_MIXED) {
            for (float **p : {&d.r32, &d.p32, &d.p32b, &d.q32, &d.x32, &d.r32b, &d.q32b}) rc = rc ? rc : dev_alloc(c, p, n3);
            rc = rc ? rc : dev_alloc(c, &d.cgi_rq, static_cast<size_t>(kRing) * kShards);
            rc = rc ? rc : dev_alloc(c, &d.cgi_qq, static_cast<size_t>(kRing) * kShards);
            rc = rc ? rc : dev_alloc(c, &d.cgi_rr, static_cast<size_t>(kMaxComp) * kRing * kShards);
            rc = rc ? rc : dev_alloc(c, &d.cgi_pq, static_cast<size_t>(kMaxComp) * kRing * kShards);
            rc = rc ? rc : dev_alloc(c, &d.cgi_bb, static_cast<size_t>(kMaxComp) * kShards);
            rc = rc ? rc : dev_alloc(c, &d.cgi_flags, 2 * kMaxComp);
            rc = rc ? rc : dev_alloc(c, &d.cgi_rz, static_cast<size_t>(kMaxComp) * kRing * kShards);
            rc = rc ? rc : dev_alloc(c, &d.cgi_rzq, static_cast<size_t>(kMaxComp) * kRing * kShards);
            rc = rc ? rc : dev_alloc(c, &d.cgi_qzq, static_cast<size_t>(kMaxComp) * kRing * kShards);
            for (int k = 0; k < 2; ++k) {
                rc = rc ? rc : dev_alloc(c, &d.gs_a32[k], nent);
                rc = rc ? rc : dev_alloc(c, &d.gs_d32[k], n);
            }
        }
        return rc;
    };
    c->arena_planning = true;
    c->arena_size = 0;
    alloc_all();
    c->arena_planning = false;
    {
        void *a = nullptr;
        rc = ctx_malloc(c, &a, c->arena_size, "device allocation (mesh arena)");
        c->arena = static_cast<char *>(a);
    }
    if (rc) {
        c->arena = nullptr;
        c->arena_size = 0;
    } else {
        c->arena_used = 0;
        rc = alloc_all();
    }
    if (rc) {
        c->release_mesh();
        return static_cast<gspm_status>(rc);
    }
    hipStream_t s = c->stream;
    hipMemcpyAsync(d.x, hm.xs.data(), sizeof(double) * n3, hipMemcpyHostToDevice, s);
    hipMemcpyAsync(d.lconn, hm.lconn.data(), sizeof(uint16_t) * hm.lconn.size(), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(d.halo_ptr, hm.halo_ptr.data(), sizeof(int32_t) * hm.halo_ptr.size(), hipMemcpyHostToDevice, s);
    if (!hm.halo_ids.empty())
        hipMemcpyAsync(d.halo_ids, hm.halo_ids.data(), sizeof(int32_t) * hm.halo_ids.size(), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(d.halo_lo, hm.halo_lo.data(), sizeof(int32_t) * hm.halo_lo.size(), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(d.img, hm.img.data(), hm.img.size(), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(d.blk_ptr, hm.blk_ptr.data(), sizeof(int32_t) * hm.blk_ptr.size(), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(d.blk_nmag, hm.blk_nmag.data(), sizeof(int32_t) * hm.blk_nmag.size(), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(d.w, hm.w.data(), sizeof(double) * n, hipMemcpyHostToDevice, s);
    hipMemcpyAsync(d.gs_off, rows.off.data(), sizeof(int32_t) * rows.off.size(), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(d.gs_halo_ptr, rows.halo_ptr.data(), sizeof(int32_t) * rows.halo_ptr.size(), hipMemcpyHostToDevice,
                   s);
    if (!rows.halo_ids.empty())
        hipMemcpyAsync(d.gs_halo_ids, rows.halo_ids.data(), sizeof(int32_t) * rows.halo_ids.size(),
                       hipMemcpyHostToDevice, s);
    if (nent) {
        hipMemcpyAsync(d.gs_col, rows.col.data(), sizeof(uint16_t) * nent, hipMemcpyHostToDevice, s);
        hipMemcpyAsync(d.gs_kv, rows.kv.data(), sizeof(double) * nent, hipMemcpyHostToDevice, s);
        hipMemcpyAsync(d.gs_mv, rows.mv.data(), sizeof(double) * nent, hipMemcpyHostToDevice, s);
    }
    hipMemcpyAsync(d.gs_kd, rows.kd.data(), sizeof(double) * n, hipMemcpyHostToDevice, s);
    hipMemcpyAsync(d.gs_md, rows.md.data(), sizeof(double) * n, hipMemcpyHostToDevice, s);
    c->gs_nent = static_cast<int64_t>(nent);
    if (c->deterministic) {
        hipMemcpyAsync(d.inc_ptr, inc_ptr.data(), sizeof(int32_t) * inc_ptr.size(), hipMemcpyHostToDevice, s);
        if (!inc_ent.empty())
            hipMemcpyAsync(d.inc_ent, inc_ent.data(), sizeof(uint16_t) * inc_ent.size(), hipMemcpyHostToDevice, s);
        const std::vector<double *> no_dst(kDetSlots, nullptr);
        hipMemcpyAsync(d.det_dst, no_dst.data(), sizeof(double *) * kDetSlots, hipMemcpyHostToDevice, s);
        launch_fill(d.det_part, static_cast<int64_t>(kDetSlots) * det_blocks, 0.0, s);
        launch_fill_i32(d.det_count, 1, 0, s);
    }
    std::vector<int32_t> rep(n, -1);
    for (int64_t i = hm.n0 - 1; i >= 0; --i) rep[static_cast<size_t>(hm.user2int[i])] = static_cast<int32_t>(i);
    hipMemcpyAsync(d.rep, rep.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s);
    if (nseg) {
        hipMemcpyAsync(d.seg_ent, hm.seg_ent.data(), sizeof(uint16_t) * hm.seg_ent.size(), hipMemcpyHostToDevice, s);
        hipMemcpyAsync(d.seg_off, hm.seg_off.data(), sizeof(uint32_t) * nseg, hipMemcpyHostToDevice, s);
        hipMemcpyAsync(d.seg_nel, hm.seg_nel.data(), sizeof(uint16_t) * nseg, hipMemcpyHostToDevice, s);
    }
    hipMemcpyAsync(d.seg_ptr, hm.seg_ptr.data(), sizeof(int32_t) * hm.seg_ptr.size(), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(d.seg_nmag, hm.seg_nmag.data(), sizeof(int32_t) * hm.seg_nmag.size(), hipMemcpyHostToDevice, s);
    for (double *p : {d.m, d.mnext, d.u, d.unext, d.ms, d.g, d.gs, d.b, d.r, d.p, d.p2, d.q, d.mprev, d.uprev, d.du_prev,
                      d.kdu})
        launch_fill(p, n3, 0.0, s);
    launch_fill(d.wcoef, 2, 0.0, s);
    launch_fill(d.ud, n, 0.0, s);
    launch_fill(d.udnext, n, 0.0, s);
    if (c->precision == GSPM_MIXED)
        for (float *p : {d.r32, d.p32, d.p32b, d.q32, d.x32}) launch_fill_f32(p, n3, s);
    launch_fill(d.ch2, 2 * n, 0.0, s);
    rc = hip_check(c, hipStreamSynchronize(s), "upload_mesh");
    if (rc) {
        c->release_mesh();
        return static_cast<gspm_status>(rc);
    }
    c->n0 = hm.n0;
    c->ne = hm.ne;
    c->ncopies = hm.ncopies;
    c->n = hm.n;
    c->nblk = hm.nblk;
    c->p0 = hm.p0;
    c->vc = hm.vc;
    for (int a = 0; a < 3; ++a) c->box_lo[a] = hm.lo[a];
    c->tets_int.resize(4 * static_cast<size_t>(n_tets));
    for (size_t q = 0; q < c->tets_int.size(); ++q) c->tets_int[q] = hm.user2int[tets[q]];
    c->user2int = std::move(hm.user2int);
    c->w_host = hm.w;
    c->nmag = 0;
    for (double wv : c->w_host) c->nmag += wv > 0.0;
    auto &mv = c->mv;
    mv.x = d.x;
    mv.y = d.x + n;
    mv.z = d.x + 2 * n;
    mv.lconn = d.lconn;
    mv.blk_ptr = d.blk_ptr;
    mv.blk_nmag = d.blk_nmag;
    mv.halo_ptr = d.halo_ptr;
    mv.halo_ids = d.halo_ids;
    mv.halo_lo = d.halo_lo;
    mv.img = d.img;
    mv.stc64 = d.stc64;
    mv.stc32 = d.stc32;
    mv.nstc = static_cast<int64_t>(static_cast<size_t>(hm.nblk) * hm.nb + hm.halo_ids.size());
    mv.seg_ent = d.seg_ent;
    mv.seg_off = d.seg_off;
    mv.seg_nel = d.seg_nel;
    mv.seg_ptr = d.seg_ptr;
    mv.seg_nmag = d.seg_nmag;
    mv.nloc_max = hm.nloc_max;
    mv.w = d.w;
    mv.n = hm.n;
    mv.nb = hm.nb;
    mv.nblk = hm.nblk;
    mv.p0 = hm.p0;
    mv.Lx = hm.L[0]; mv.Ly = hm.L[1]; mv.Lz = hm.L[2];
    mv.iLx = 1.0 / hm.L[0]; mv.iLy = 1.0 / hm.L[1]; mv.iLz = 1.0 / hm.L[2];
    mv.len_scale = std::cbrt(hm.vc / static_cast<double>(hm.ne));
    mv.det = DetSums{};
    mv.inc_ptr = nullptr;
    mv.inc_ent = nullptr;
    if (c->deterministic) {
        mv.det = DetSums{d.det_part, d.det_dst, d.det_count, det_blocks};
        mv.inc_ptr = d.inc_ptr;
        mv.inc_ent = d.inc_ent;
    }
    c->cg.det = mv.det;
    c->cg_in.det = mv.det;
    c->mv_rows = mv;
    c->mv_rows.nb = rows.nb;
    c->mv_rows.nblk = rows.nblk;
    c->mv_rows.halo_ptr = d.gs_halo_ptr;
    c->mv_rows.halo_ids = d.gs_halo_ids;
    c->mv_rows.nloc_max = rows.nloc_max;
    c->cg.rr = d.cg_rr;
    c->cg.pq = d.cg_pq;
    c->cg.bb = d.cg_bb;
    c->cg.rq = d.cg_rq;
    c->cg.qq = d.cg_qq;
    c->cg.rz = d.cg_rz;
    c->cg.rzq = d.cg_rzq;
    c->cg.qzq = d.cg_qzq;
    c->cg.done = d.cg_flags;
    c->cg.iters = d.cg_flags + kMaxComp;
    c->cg.ring = kRing;
    c->cg_in.rr = d.cgi_rr;
    c->cg_in.pq = d.cgi_pq;
    c->cg_in.bb = d.cgi_bb;
    c->cg_in.rq = d.cgi_rq;
    c->cg_in.qq = d.cgi_qq;
    c->cg_in.rz = d.cgi_rz;
    c->cg_in.rzq = d.cgi_rzq;
    c->cg_in.qzq = d.cgi_qzq;
    c->cg_in.done = d.cgi_flags;
    c->cg_in.iters = d.cgi_flags ? d.cgi_flags + kMaxComp : nullptr;
    c->cg_in.ring = kRing;
    c->dargs.vc = hm.vc;
    launch_stage_coords(mv, d.stc64, d.stc32, c->stream);
    rc = hip_check(c, hipStreamSynchronize(c->stream), "upload_mesh");
    if (rc) {
        c->release_mesh();
        return static_cast<gspm_status>(rc);
    }
    c->have_mesh = true;
    c->have_m = false;
    return GSPM_OK;
}

gspm_status gspm_set_gs_start(gspm_ctx *c, int32_t mode) {
    if (!c) return GSPM_E_ARG;
    if (mode != GSPM_GS_START_LUMPED && mode != GSPM_GS_START_CORRECTED)
        return fail(c, GSPM_E_ARG, "set_gs_start: unknown mode");
    if (mode == GSPM_GS_START_CORRECTED && c->deterministic)
        return fail(c, GSPM_E_STATE, "the corrected GS start is not available in deterministic mode");
    if (mode != c->gs_start) c->gcorr_ok = 0;
    c->gs_start = mode;
    return GSPM_OK;
}

gspm_status gspm_set_params(gspm_ctx *c, const gspm_params *p) {
    if (!c) return GSPM_E_ARG;
    if (!p) return fail(c, GSPM_E_ARG, "set_params: null params");
    if (!c->have_mesh) return fail(c, GSPM_E_STATE, "set_params before upload_mesh");
    const double *raw = &p->Ms;
    if (!all_finite(raw, 11) || !all_finite(p->Nd, 9) || !all_finite(p->hext, 3) || !all_finite(p->sigma_ext, 6) ||
        !std::isfinite(p->cg_tol))
        return fail(c, GSPM_E_ARG, "set_params: non-finite value");
    if (!(p->Ms > 0 && p->A >= 0 && p->mu0 > 0 && p->gamma0 > 0 && p->alpha >= 0 && p->cg_tol > 0 && p->cg_maxit > 0))
        return fail(c, GSPM_E_ARG, "set_params: Ms, mu0, gamma0, cg_tol, cg_maxit must be positive; A, alpha >= 0");
    if (!(p->c44 > 0 && p->c11 - p->c12 > 0 && p->c11 + 2 * p->c12 > 0))
        return fail(c, GSPM_E_ARG, "set_params: elastic constants are not positive definite");
    if (p->local_demag != 0 && p->local_demag != 1) return fail(c, GSPM_E_ARG, "set_params: local_demag must be 0 or 1");
    if (p->elastic_precond != GSPM_PRECOND_NONE && p->elastic_precond != GSPM_PRECOND_GREEN)
        return fail(c, GSPM_E_ARG, "set_params: unknown elastic_precond");
    if (!(p->ms_tol >= 0.0) || !std::isfinite(p->ms_tol)) return fail(c, GSPM_E_ARG, "set_params: ms_tol must be >= 0");
    if (p->gs_precond != GSPM_PRECOND_NONE && p->gs_precond != GSPM_PRECOND_JACOBI)
        return fail(c, GSPM_E_ARG, "set_params: gs_precond must be GSPM_PRECOND_NONE or GSPM_PRECOND_JACOBI");
    double R[9];
    bool zero = true, ident = true;
    for (int k = 0; k < 9; ++k) {
        zero &= p->crystal_rot[k] == 0.0;
        ident &= p->crystal_rot[k] == ((k % 4 == 0) ? 1.0 : 0.0);
    }
    for (int k = 0; k < 9; ++k) R[k] = zero ? ((k % 4 == 0) ? 1.0 : 0.0) : p->crystal_rot[k];
    if (!all_finite(R, 9)) return fail(c, GSPM_E_ARG, "set_params: non-finite crystal_rot");
    {
        double err = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                err = std::max(err, std::fabs(R[3 * i] * R[3 * j] + R[3 * i + 1] * R[3 * j + 1] +
                                              R[3 * i + 2] * R[3 * j + 2] - (i == j ? 1.0 : 0.0)));
        const double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                           R[2] * (R[3] * R[7] - R[4] * R[6]);
        if (!(err < 1e-12) || !(det > 0.0)) return fail(c, GSPM_E_ARG, "set_params: crystal_rot is not a proper rotation");
    }
    c->p = *p;
    auto &m = c->mat;
    m.c11 = p->c11; m.c12 = p->c12; m.c44 = p->c44;
    m.l100 = p->lambda100; m.l111 = p->lambda111;
    m.kan = 2.0 * p->K1 / (p->mu0 * p->Ms * p->Ms);
    m.kme = 1.0 / (p->mu0 * p->Ms * p->Ms);
    m.A = p->A; m.K1 = p->K1; m.mu0Ms = p->mu0 * p->Ms;
    m.rot = (zero || ident) ? 0 : 1;
    for (int k = 0; k < 9; ++k) m.R[k] = R[k];
    sample_stiffness(*p, R, m.C6);
    c->dargs.rot = m.rot;
    for (int k = 0; k < 9; ++k) c->dargs.R[k] = R[k];
    for (int k = 0; k < 9; ++k) c->dargs.Nd[k] = p->Nd[k];
    for (int k = 0; k < 3; ++k) c->dargs.hz[k] = p->hext[k] / p->Ms;
    {
        // C^-1 sigma_ext in the crystal frame, carried back: R (C^-1 (R^T sigma R)) R^T
        double sc[6], ec[6];
        rotate_sym(R, false, p->sigma_ext, sc);
        cubic_compliance(*p, sc, ec);
        rotate_sym(R, true, ec, c->dargs.csig);
    }
    c->have_params = true;
    if (p->elastic_precond == GSPM_PRECOND_GREEN) {
        hipSetDevice(c->device);
        const int rc = green_setup(c);
        if (rc) {
            c->p.elastic_precond = GSPM_PRECOND_NONE;
            return static_cast<gspm_status>(rc);
        }
    }
    return GSPM_OK;
}

gspm_status gspm_set_field(gspm_ctx *c, gspm_field which, const double *v, int64_t n_nodes) {
    if (!c) return GSPM_E_ARG;
    if (!v) return fail(c, GSPM_E_ARG, "set_field: null array");
    if (!c->have_mesh) return fail(c, GSPM_E_STATE, "set_field before upload_mesh");
    if (n_nodes != c->n0) return fail(c, GSPM_E_ARG, "set_field: node count differs from the mesh");
    if (which != GSPM_FIELD_M && which != GSPM_FIELD_U && which != GSPM_FIELD_UD)
        return fail(c, GSPM_E_ARG, "set_field: unknown field");
    hipSetDevice(c->device);
    std::vector<double> h;
    if (which == GSPM_FIELD_UD) {
        // one value per node: spread into the first column of the n0 x 3 layout
        std::vector<double> v3(3 * static_cast<size_t>(c->n0), 0.0);
        for (int64_t i = 0; i < c->n0; ++i) v3[3 * i] = v[i];
        int rc = gather_user(c, v3.data(), h);
        if (rc) return static_cast<gspm_status>(rc);
        h.resize(static_cast<size_t>(c->n));
        return static_cast<gspm_status>(upload(c, c->d.ud, h));
    }
    int rc = gather_user(c, v, h);
    if (rc) return static_cast<gspm_status>(rc);
    const int n = c->n;
    if (which == GSPM_FIELD_M) {
        for (int k = 0; k < n; ++k) {
            double *a = &h[k], *b = &h[static_cast<size_t>(n) + k], *cc = &h[2 * static_cast<size_t>(n) + k];
            if (!(c->w_host[k] > 0.0)) {
                *a = *b = *cc = 0.0;
                continue;
            }
            const double r = std::sqrt(*a * *a + *b * *b + *cc * *cc);
            if (!(r > 0.0)) return fail(c, GSPM_E_ARG, "set_field: zero magnetisation on a magnetic node");
            // a vector of unit length to rounding (a state read back with get_field) is kept bit for bit,
            // so a saved state restores exactly
            if (std::fabs(r - 1.0) > 1e-14) {
                *a /= r; *b /= r; *cc /= r;
            }
        }
        rc = upload(c, c->d.m, h);
        if (rc) return static_cast<gspm_status>(rc);
        c->have_m = true;
        c->have_prev = false;     // a new state has no history for the warm starts
        c->gcorr_ok = 0;
        c->commits = 0;
    } else {
        rc = upload(c, c->d.u, h);
        if (rc) return static_cast<gspm_status>(rc);
        c->commits = 0;           // u^{n-2} no longer precedes u
    }
    return GSPM_OK;
}

gspm_status gspm_get_field(gspm_ctx *c, gspm_field which, double *out, int64_t n_nodes) {
    if (!c) return GSPM_E_ARG;
    if (!out) return fail(c, GSPM_E_ARG, "get_field: null array");
    if (!c->have_mesh) return fail(c, GSPM_E_STATE, "get_field before upload_mesh");
    if (n_nodes != c->n0) return fail(c, GSPM_E_ARG, "get_field: node count differs from the mesh");
    if (which != GSPM_FIELD_M && which != GSPM_FIELD_U && which != GSPM_FIELD_UD)
        return fail(c, GSPM_E_ARG, "get_field: unknown field");
    hipSetDevice(c->device);
    if (which == GSPM_FIELD_UD) {
        std::vector<double> h(static_cast<size_t>(c->n));
        int rc = download(c, c->d.ud, h);
        if (rc) return static_cast<gspm_status>(rc);
        for (int64_t i = 0; i < c->n0; ++i) out[i] = h[static_cast<size_t>(c->user2int[i])];
        return GSPM_OK;
    }
    std::vector<double> h(3 * static_cast<size_t>(c->n));
    int rc = download(c, which == GSPM_FIELD_M ? c->d.m : c->d.u, h);
    if (rc) return static_cast<gspm_status>(rc);
    scatter_user(c, h, out);
    return GSPM_OK;
}

gspm_status gspm_step(gspm_ctx *c, double dt, int32_t n_steps, gspm_step_stats *stats) {
    if (!c) return GSPM_E_ARG;
    if (!c->have_mesh || !c->have_params || !c->have_m)
        return fail(c, GSPM_E_STATE, "step needs upload_mesh, set_params and set_field(M) first");
    if (!(dt > 0) || !std::isfinite(dt) || n_steps < 0) return fail(c, GSPM_E_ARG, "step: dt must be positive, n >= 0");
    hipSetDevice(c->device);
    gspm_step_stats local;
    gspm_step_stats *st = stats ? stats : &local;
    return static_cast<gspm_status>(run_steps(c, dt, n_steps, st));
}

gspm_status gspm_energies(gspm_ctx *c, double out[7]) {
    if (!c) return GSPM_E_ARG;
    if (!out) return fail(c, GSPM_E_ARG, "energies: null output");
    if (!c->have_mesh || !c->have_params || !c->have_m) return fail(c, GSPM_E_STATE, "energies need mesh, params and m");
    hipSetDevice(c->device);
    auto &d = c->d;
    hipStream_t s = c->stream;
    launch_avg_sums(c->n, d.w, d.m, c->mat, d.sums, s, c->mv.det);
    launch_derive(d.sums, c->dargs, &d.der[0], s);
    launch_fill(d.esums, 5 * kShards, 0.0, s);
    launch_energy_elem(c->mv, c->mat, d.m, d.u, c->p.local_demag ? d.ud : nullptr, &d.der[0], d.esums, s);
    launch_energy_nodes(c->n, d.w, d.m, c->mat, c->p.hext, d.esums + 2 * kShards, s, c->mv.det);
    double es[5 * kShards];
    Derived der;
    hipMemcpyAsync(es, d.esums, sizeof es, hipMemcpyDeviceToHost, s);
    hipMemcpyAsync(&der, &d.der[0], sizeof der, hipMemcpyDeviceToHost, s);
    int rc = hip_check(c, hipStreamSynchronize(s), "energies");
    if (rc) return static_cast<gspm_status>(rc);
    double tot[4] = {0, 0, 0, 0};
    for (int k = 0; k < 4; ++k)
        for (int q = 0; q < kShards; ++q) tot[k] += es[k * kShards + q];
    const gspm_params &p = c->p;
    out[0] = tot[0] / c->vc;
    out[1] = tot[2] / c->vc;
    out[2] = tot[3] / c->vc;
    out[3] = tot[1] / c->vc;
    const double *sg = p.sigma_ext, *eb = der.ebar;
    out[4] = -(sg[0] * eb[0] + sg[1] * eb[1] + sg[2] * eb[2] + 2.0 * (sg[3] * eb[3] + sg[4] * eb[4] + sg[5] * eb[5]));
    double dem = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) dem += der.mbar[a] * p.Nd[a * 3 + b] * der.mbar[b];
    out[5] = 0.5 * p.mu0 * p.Ms * p.Ms * dem;
    out[6] = out[0] + out[1] + out[2] + out[3] + out[4] + out[5];
    if (p.local_demag) {
        double dl = 0.0;
        for (int q = 0; q < kShards; ++q) dl += es[4 * kShards + q];
        out[6] += 0.5 * p.mu0 * dl / c->vc;
    }
    return GSPM_OK;
}

gspm_status gspm_demag_local_energy(gspm_ctx *c, double *e) {
    if (!c) return GSPM_E_ARG;
    if (!e) return fail(c, GSPM_E_ARG, "demag_local_energy: null output");
    if (!c->have_mesh || !c->have_params || !c->have_m)
        return fail(c, GSPM_E_STATE, "demag_local_energy needs mesh, params and m");
    hipSetDevice(c->device);
    auto &d = c->d;
    hipStream_t s = c->stream;
    // the element pass also needs m, u and the averages; only its potential sum is used here
    launch_avg_sums(c->n, d.w, d.m, c->mat, d.sums, s, c->mv.det);
    launch_derive(d.sums, c->dargs, &d.der[0], s);
    launch_fill(d.esums, 5 * kShards, 0.0, s);
    launch_energy_elem(c->mv, c->mat, d.m, d.u, d.ud, &d.der[0], d.esums, s);
    double es[kShards];
    hipMemcpyAsync(es, d.esums + 4 * kShards, sizeof es, hipMemcpyDeviceToHost, s);
    int rc = hip_check(c, hipStreamSynchronize(s), "demag_local_energy");
    if (rc) return static_cast<gspm_status>(rc);
    double dl = 0.0;
    for (int q = 0; q < kShards; ++q) dl += es[q];
    *e = 0.5 * c->p.mu0 * dl / c->vc;
    return GSPM_OK;
}

gspm_status gspm_averages(gspm_ctx *c, double mbar[3], double ebar[6]) {
    if (!c) return GSPM_E_ARG;
    if (!mbar || !ebar) return fail(c, GSPM_E_ARG, "averages: null output");
    if (!c->have_mesh || !c->have_params || !c->have_m) return fail(c, GSPM_E_STATE, "averages need mesh, params and m");
    hipSetDevice(c->device);
    launch_avg_sums(c->n, c->d.w, c->d.m, c->mat, c->d.sums, c->stream, c->mv.det);
    launch_derive(c->d.sums, c->dargs, &c->d.der[0], c->stream);
    Derived der;
    hipMemcpyAsync(&der, &c->d.der[0], sizeof der, hipMemcpyDeviceToHost, c->stream);
    int rc = hip_check(c, hipStreamSynchronize(c->stream), "averages");
    if (rc) return static_cast<gspm_status>(rc);
    for (int k = 0; k < 3; ++k) mbar[k] = der.mbar[k];
    for (int k = 0; k < 6; ++k) ebar[k] = der.ebar[k];
    return GSPM_OK;
}

gspm_status gspm_averages_noalloc(gspm_ctx *c, const double *m_dev, double *out_dev) {
    if (!c) return GSPM_E_ARG;
    if (!m_dev || !out_dev) return fail(c, GSPM_E_ARG, "averages_noalloc: null device pointer");
    if (!c->have_mesh || !c->have_params) return fail(c, GSPM_E_STATE, "averages_noalloc needs mesh and params");
    if (c->n > kNaMaxNodes)
        return fail(c, GSPM_E_ARG, "averages_noalloc: " + std::to_string(c->n) + " unique nodes, more than the " +
                                       std::to_string(kNaMaxNodes) + " its fixed scratch serves");
    hipSetDevice(c->device);
    const int e = launch_averages_noalloc(c->na_scratch, c->n, c->d.w, c->d.rep, m_dev, c->mat, c->dargs, out_dev,
                                          c->stream);
    if (e != 0) return fail(c, GSPM_E_DEVICE, std::string("averages_noalloc: ") +
                                                  hipGetErrorString(static_cast<hipError_t>(e)));
    return GSPM_OK;
}

gspm_status gspm_apply(gspm_ctx *c, gspm_op op, double eps, const double *x, double *y, int64_t n_nodes) {
    if (!c) return GSPM_E_ARG;
    if (!x || !y) return fail(c, GSPM_E_ARG, "apply: null array");
    if (!c->have_mesh) return fail(c, GSPM_E_STATE, "apply before upload_mesh");
    if (n_nodes != c->n0) return fail(c, GSPM_E_ARG, "apply: node count differs from the mesh");
    if (op < GSPM_OP_LAPLACE || op > GSPM_OP_PRECOND) return fail(c, GSPM_E_ARG, "apply: unknown operator");
    if (op == GSPM_OP_ELASTIC && !c->have_params) return fail(c, GSPM_E_STATE, "apply(ELASTIC) needs set_params");
    if (op == GSPM_OP_PRECOND &&
        !(c->have_params && c->p.elastic_precond == GSPM_PRECOND_GREEN && c->precision == GSPM_FP64))
        return fail(c, GSPM_E_STATE, "apply(PRECOND) needs elastic_precond = GSPM_PRECOND_GREEN on an FP64 context");
    if (!std::isfinite(eps)) return fail(c, GSPM_E_ARG, "apply: non-finite eps");
    hipSetDevice(c->device);
    std::vector<double> h;
    int rc = gather_user(c, x, h);
    if (rc) return static_cast<gspm_status>(rc);
    rc = upload(c, c->d.ms, h);
    if (rc) return static_cast<gspm_status>(rc);
    if (op == GSPM_OP_PRECOND) {
        rc = green_apply64(c, c->d.ms, c->d.q);
        if (rc) return static_cast<gspm_status>(rc);
    } else if (op == GSPM_OP_ELASTIC) {
        launch_elastic_matvec<double>(c->mv, c->mat, MV_APPLY, c->d.ms, c->d.q, nullptr, nullptr, nullptr, c->cg, 0,
                                      0.0, c->stream);
    } else if (op == GSPM_OP_MS) {
        launch_ms_matvec<double>(c->mv, 3, MV_APPLY, c->d.ms, c->d.q, nullptr, nullptr, nullptr, c->cg, 0, 0.0,
                                 c->stream);
    } else {
        const double e = op == GSPM_OP_LAPLACE ? 1.0 : (op == GSPM_OP_MASS ? 0.0 : eps);
        const double mass = op == GSPM_OP_LAPLACE ? 0.0 : 1.0;
        launch_gs_rows<double>(c->mv_rows, gs_rows(c, e, mass, false), 3, MV_APPLY, c->d.ms, c->d.q, nullptr, nullptr,
                               c->cg, c->stream);
    }
    rc = download(c, c->d.q, h);
    if (rc) return static_cast<gspm_status>(rc);
    scatter_user(c, h, y);
    return GSPM_OK;
}

gspm_status gspm_solve(gspm_ctx *c, gspm_op op, double eps, const double *b, double *x, int64_t n_nodes, double tol,
                       int32_t maxit, int32_t *iters) {
    if (!c) return GSPM_E_ARG;
    if (!b || !x) return fail(c, GSPM_E_ARG, "solve: null array");
    if (!c->have_mesh) return fail(c, GSPM_E_STATE, "solve before upload_mesh");
    if (n_nodes != c->n0) return fail(c, GSPM_E_ARG, "solve: node count differs from the mesh");
    if (op != GSPM_OP_GS && op != GSPM_OP_ELASTIC && op != GSPM_OP_MS)
        return fail(c, GSPM_E_ARG, "solve: operator must be GS, ELASTIC or MS");
    if (op == GSPM_OP_ELASTIC && !c->have_params) return fail(c, GSPM_E_STATE, "solve(ELASTIC) needs set_params");
    if (!(tol > 0) || maxit <= 0 || !std::isfinite(eps)) return fail(c, GSPM_E_ARG, "solve: tol and maxit must be positive");
    hipSetDevice(c->device);
    std::vector<double> hb, hx;
    int rc = gather_user(c, b, hb);
    if (!rc) rc = gather_user(c, x, hx);
    if (rc) return static_cast<gspm_status>(rc);
    const int n = c->n;
    const bool el = op == GSPM_OP_ELASTIC, msop = op == GSPM_OP_MS;
    const int ns = el ? 1 : 3;
    const bool green = el && c->p.elastic_precond == GSPM_PRECOND_GREEN;
    for (int k = 0; k < n; ++k) {
        if (green) break;              // the periodic system: nothing pinned before the solve
        const bool fixed = (el || msop) ? (k == c->p0) : !(c->w_host[k] > 0.0);
        if (!fixed) continue;
        for (int a = 0; a < 3; ++a) hb[static_cast<size_t>(a) * n + k] = hx[static_cast<size_t>(a) * n + k] = 0.0;
    }
    std::vector<double> bbh(static_cast<size_t>(kMaxComp) * kShards, 0.0);
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < n; ++k) bbh[static_cast<size_t>(el ? 0 : a) * kShards] += hb[static_cast<size_t>(a) * n + k] * hb[static_cast<size_t>(a) * n + k];
    cg_prepare(c, ns);
    hipMemcpyAsync(c->d.cg_bb, bbh.data(), sizeof(double) * bbh.size(), hipMemcpyHostToDevice, c->stream);
    rc = upload(c, c->d.b, hb);
    if (!rc) rc = upload(c, c->d.mnext, hx);
    if (rc) return static_cast<gspm_status>(rc);
    CgResult r = el ? cg_elastic(c, c->d.mnext, c->d.b, tol, maxit, SK_OTHER)
                 : msop ? cg_ms(c, 3, c->d.mnext, c->d.b, tol, maxit, SK_OTHER)
                        : cg_gs(c, 3, eps, c->d.mnext, c->d.b, tol, maxit, SK_OTHER);
    if (iters) *iters = r.iters[0] + r.iters[1] + r.iters[2];
    rc = download(c, c->d.mnext, hx);
    if (rc) return static_cast<gspm_status>(rc);
    scatter_user(c, hx, x);
    return static_cast<gspm_status>(r.status);
}

gspm_status gspm_time_operator(gspm_ctx *c, gspm_op op, double eps, int32_t reps, double *avg_ms) {
    if (!c) return GSPM_E_ARG;
    if (!avg_ms || reps <= 0 || !std::isfinite(eps)) return fail(c, GSPM_E_ARG, "time_operator: bad arguments");
    if (!c->have_mesh) return fail(c, GSPM_E_STATE, "time_operator before upload_mesh");
    if (op < GSPM_OP_LAPLACE || op > GSPM_OP_MS) return fail(c, GSPM_E_ARG, "time_operator: unknown operator");
    if (op == GSPM_OP_ELASTIC && !c->have_params) return fail(c, GSPM_E_STATE, "time_operator(ELASTIC) needs set_params");
    hipSetDevice(c->device);
    const double e = op == GSPM_OP_LAPLACE ? 1.0 : (op == GSPM_OP_MASS ? 0.0 : eps);
    const double mass = op == GSPM_OP_LAPLACE ? 0.0 : 1.0;
    const bool f32 = c->precision == GSPM_MIXED;   // time the operator the inner solves use
    const bool gsop = op != GSPM_OP_ELASTIC && op != GSPM_OP_MS;
    const GsRowsView rv = gsop ? gs_rows(c, e, mass, f32) : GsRowsView{};
    hipEventRecord(c->t0, c->stream);
    for (int i = 0; i < reps; ++i) {
        if (op == GSPM_OP_ELASTIC) {
            if (f32)
                launch_elastic_matvec<float>(c->mv, c->mat, MV_APPLY, c->d.r32, c->d.q32, nullptr, nullptr, nullptr,
                                             c->cg, 0, 0.0, c->stream);
            else
                launch_elastic_matvec<double>(c->mv, c->mat, MV_APPLY, c->d.ms, c->d.q, nullptr, nullptr, nullptr,
                                              c->cg, 0, 0.0, c->stream);
        } else if (op == GSPM_OP_MS) {
            // one component, as the step's solve
            if (f32)
                launch_ms_matvec<float>(c->mv, 1, MV_APPLY, c->d.r32, c->d.q32, nullptr, nullptr, nullptr, c->cg, 0,
                                        0.0, c->stream);
            else
                launch_ms_matvec<double>(c->mv, 1, MV_APPLY, c->d.ms, c->d.q, nullptr, nullptr, nullptr, c->cg, 0,
                                         0.0, c->stream);
        } else {
            if (f32)
                launch_gs_rows<float>(c->mv_rows, rv, 3, MV_APPLY, c->d.r32, c->d.q32, nullptr, nullptr, c->cg, c->stream);
            else
                launch_gs_rows<double>(c->mv_rows, rv, 3, MV_APPLY, c->d.ms, c->d.q, nullptr, nullptr, c->cg, c->stream);
        }
    }
    hipEventRecord(c->t1, c->stream);
    int rc = hip_check(c, hipEventSynchronize(c->t1), "time_operator");
    if (rc) return static_cast<gspm_status>(rc);
    float ms = 0.0f;
    hipEventElapsedTime(&ms, c->t0, c->t1);
    *avg_ms = ms / reps;
    return GSPM_OK;
}

gspm_status gspm_set_profile(gspm_ctx *c, int32_t enable) {
    if (!c) return GSPM_E_ARG;
    c->profile = enable != 0;
    return GSPM_OK;
}

gspm_status gspm_mesh_info(gspm_ctx *c, int64_t *n_unique, int64_t *n_tets, int64_t *n_blocks, int64_t *n_copies,
                           double *volume) {
    if (!c) return GSPM_E_ARG;
    if (!c->have_mesh) return fail(c, GSPM_E_STATE, "mesh_info before upload_mesh");
    if (n_unique) *n_unique = c->n;
    if (n_tets) *n_tets = c->ne;
    if (n_blocks) *n_blocks = c->nblk;
    if (n_copies) *n_copies = c->ncopies;
    if (volume) *volume = c->vc;
    return GSPM_OK;
}

gspm_status gspm_demag_factors(double a, double b, double c, double N[3]) {
    if (!N || !(a > 0) || !(b > 0) || !(c > 0) || !std::isfinite(a) || !std::isfinite(b) || !std::isfinite(c))
        return GSPM_E_ARG;
    demag_factors(a, b, c, N);
    return GSPM_OK;
}

const char *gspm_last_error(const gspm_ctx *c) { return c ? c->err.c_str() : g_create_error.c_str(); }

}  // extern "C"
