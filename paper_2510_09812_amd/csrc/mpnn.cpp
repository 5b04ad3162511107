// Learned elastic warm start: host side (graph construction, device state,
// the C ABI entry points and the start used by the time step).  All network
// arithmetic runs in the kernels of mpnn.hip.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "context.h"

namespace gspm {
namespace mpnn {

void build_edge_graph(int32_t n, const std::vector<int32_t> &tets, std::vector<int32_t> &ptr,
                      std::vector<int32_t> &nbr) {
    const size_t ne = tets.size() / 4;
    std::vector<int32_t> inc_ptr(static_cast<size_t>(n) + 1, 0), inc;
    for (int32_t v : tets) ++inc_ptr[static_cast<size_t>(v) + 1];
    for (int32_t i = 0; i < n; ++i) inc_ptr[i + 1] += inc_ptr[i];
    inc.resize(tets.size());
    {
        std::vector<int32_t> fill(inc_ptr.begin(), inc_ptr.end() - 1);
        for (size_t e = 0; e < ne; ++e)
            for (int k = 0; k < 4; ++k) inc[fill[tets[4 * e + k]]++] = static_cast<int32_t>(e);
    }
    ptr.assign(static_cast<size_t>(n) + 1, 0);
    nbr.clear();
    nbr.reserve(static_cast<size_t>(n) * 16);
    std::vector<int32_t> tmp;
    for (int32_t i = 0; i < n; ++i) {
        tmp.clear();
        for (int32_t q = inc_ptr[i]; q < inc_ptr[i + 1]; ++q) {
            const size_t e = static_cast<size_t>(inc[q]);
            for (int k = 0; k < 4; ++k) {
                const int32_t v = tets[4 * e + k];
                if (v != i) tmp.push_back(v);
            }
        }
        std::sort(tmp.begin(), tmp.end());
        tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
        nbr.insert(nbr.end(), tmp.begin(), tmp.end());
        ptr[static_cast<size_t>(i) + 1] = static_cast<int32_t>(nbr.size());
    }
}

}  // namespace mpnn

namespace {

template <class T>
int nn_alloc(gspm_ctx *c, T **p, size_t count) {
    void *v = nullptr;
    const int rc = ctx_malloc(c, &v, sizeof(T) * std::max<size_t>(count, 1), "device allocation (network)");
    *p = static_cast<T *>(v);
    return rc;
}

gspm_status nfail(gspm_ctx *c, gspm_status s, const char *msg) {
    c->err = msg;
    return s;
}

// Graph, weights and activation buffers, built on first use after a mesh upload.
int nn_setup(gspm_ctx *c) {
    auto &nn = c->nn;
    if (nn.ready) return GSPM_OK;
    using namespace mpnn;
    std::vector<int32_t> ptr, nbr;
    build_edge_graph(c->n, c->tets_int, ptr, nbr);
    const size_t n = static_cast<size_t>(c->n);
    int rc = 0;
    rc = rc ? rc : nn_alloc(c, &nn.gptr, ptr.size());
    rc = rc ? rc : nn_alloc(c, &nn.gnbr, nbr.size());
    rc = rc ? rc : nn_alloc(c, &nn.master, kNParam);
    rc = rc ? rc : nn_alloc(c, &nn.wr, kNParam);
    rc = rc ? rc : nn_alloc(c, &nn.m1, kNParam);
    rc = rc ? rc : nn_alloc(c, &nn.m2, kNParam);
    rc = rc ? rc : nn_alloc(c, &nn.grad, kNParam);
    rc = rc ? rc : nn_alloc(c, &nn.mats, static_cast<size_t>(kLayers) * 4 * kMat);
    rc = rc ? rc : nn_alloc(c, &nn.acts, n * kHid * (kLayers + 1) + n * 128 * kLayers + n * kHid * kLayers);
    rc = rc ? rc : nn_alloc(c, &nn.y, 3 * n);
    rc = rc ? rc : nn_alloc(c, &nn.red, static_cast<size_t>(R_COUNT) * kShards);
    rc = rc ? rc : nn_alloc(c, &nn.dvec, 3 * n);
    rc = rc ? rc : nn_alloc(c, &nn.du, 3 * n);
    rc = rc ? rc : nn_alloc(c, &nn.mp_in, 3 * n);
    rc = rc ? rc : nn_alloc(c, &nn.m_in, 3 * n);
    rc = rc ? rc : nn_alloc(c, &nn.gh, n * kHid);
    rc = rc ? rc : nn_alloc(c, &nn.gha, n * 128);
    rc = rc ? rc : nn_alloc(c, &nn.gab, n * 128);
    rc = rc ? rc : nn_alloc(c, &nn.gy, 3 * n);
    nn.part_wgs = static_cast<int>(std::min<size_t>(512, std::max<size_t>(1, (n + 255) / 256)));
    rc = rc ? rc : nn_alloc(c, &nn.part, static_cast<size_t>(nn.part_wgs) * kPartStride);
    if (rc) {
        c->release_nn();
        return rc;
    }
    hipStream_t s = c->stream;
    hipMemcpyAsync(nn.gptr, ptr.data(), sizeof(int32_t) * ptr.size(), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(nn.gnbr, nbr.data(), sizeof(int32_t) * std::max<size_t>(nbr.size(), 1), hipMemcpyHostToDevice, s);
    rc = hip_check(c, hipStreamSynchronize(s), "network setup");
    if (rc) {
        c->release_nn();
        return rc;
    }
    nn.nedges = static_cast<int64_t>(nbr.size());
    // mean spacing: the edge of a cube split into 6 tetrahedra of the mean volume
    const double hbar = std::cbrt(6.0 * c->vc / static_cast<double>(c->ne));
    nn.graph = Graph{nn.gptr, nn.gnbr, c->n, static_cast<float>(1.0 / hbar)};
    nn.net = Net{nn.wr, nn.mats};
    uint16_t *a = nn.acts;
    for (int l = 0; l <= kLayers; ++l, a += n * kHid) nn.A.H[l] = a;
    for (int l = 0; l < kLayers; ++l, a += n * 128) nn.A.AB[l] = a;
    for (int l = 0; l < kLayers; ++l, a += n * kHid) nn.A.AGG[l] = a;
    nn.A.y = nn.y;
    nn.G = Grads{nn.gh, nn.gha, nn.gab, nn.gy, nn.part, nn.part_wgs};
    nn.ready = true;
    return GSPM_OK;
}

}  // namespace

int minres_start(gspm_ctx *c, const double *m, const double *mprev, const double *uprev, double *x, const double *b) {
    auto &nn = c->nn;
    auto &d = c->d;
    hipStream_t s = c->stream;
    const double *dv = nullptr, *ev = nullptr;
    if (mprev) {
        mpnn::launch_forward(nn.graph, c->mv, nn.net, m, mprev, nn.red, nn.A, c->mat.l100, nn.dvec, s);
        launch_elastic_matvec<double>(c->mv, c->mat, MV_APPLY, nn.dvec, d.q, nullptr, nullptr, nullptr, c->cg, 0, 0.0,
                                      s);
        dv = nn.dvec;
    }
    if (uprev) {
        mpnn::launch_sub(3 * static_cast<int64_t>(c->n), x, uprev, d.du_prev, s);
        launch_elastic_matvec<double>(c->mv, c->mat, MV_APPLY, d.du_prev, d.kdu, nullptr, nullptr, nullptr, c->cg, 0,
                                      0.0, s);
        ev = d.du_prev;
    }
    launch_elastic_matvec<double>(c->mv, c->mat, MV_RESID, x, nullptr, b, d.r, nullptr, c->cg, 0, 0.0, s);
    mpnn::launch_minres(c->n, dv, d.q, ev, d.kdu, d.r, x, d.wred, d.wcoef, s);
    launch_zero_ring(c->cg, 1, 0, 1, 0, 0, s);
    return GSPM_OK;
}

}  // namespace gspm

using namespace gspm;

namespace {

// Caller-order fields -> internal device vectors (via the context's gather).
int upload_user(gspm_ctx *c, const double *v, double *dst) {
    std::vector<double> h;
    int rc = gather_user(c, v, h);
    if (rc) return rc;
    rc = hip_check(c, hipMemcpyAsync(dst, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, c->stream),
                   "copy to device");
    return rc ? rc : hip_check(c, hipStreamSynchronize(c->stream), "copy to device");
}

gspm_status nn_ready(gspm_ctx *c) {
    if (!c->have_mesh) return nfail(c, GSPM_E_STATE, "network call before upload_mesh");
    if (!c->nn.have_params) return nfail(c, GSPM_E_STATE, "network call before gspm_mpnn_set_params");
    return GSPM_OK;
}

}  // namespace

extern "C" {

gspm_status gspm_set_warm_start(gspm_ctx *c, int32_t mode) {
    if (!c) return GSPM_E_ARG;
    if (mode != GSPM_WARM_PREVIOUS && mode != GSPM_WARM_LEARNED && mode != GSPM_WARM_EXTRAPOLATE)
        return nfail(c, GSPM_E_ARG, "unknown warm start");
    if (mode == GSPM_WARM_LEARNED && !c->nn.have_params)
        return nfail(c, GSPM_E_STATE, "learned warm start needs gspm_mpnn_set_params");
    if (mode != GSPM_WARM_PREVIOUS && c->deterministic)
        return nfail(c, GSPM_E_STATE, "the learned and extrapolated warm starts are not available in deterministic mode");
    c->warm_mode = mode;
    return GSPM_OK;
}

gspm_status gspm_mpnn_set_params(gspm_ctx *c, const float *params, int64_t count) {
    if (!c) return GSPM_E_ARG;
    if (!params || count != mpnn::kNParam) return nfail(c, GSPM_E_ARG, "mpnn_set_params: need GSPM_MPNN_PARAMS floats");
    for (int64_t j = 0; j < count; ++j)
        if (!std::isfinite(params[j])) return nfail(c, GSPM_E_ARG, "mpnn_set_params: non-finite parameter");
    if (!c->have_mesh) return nfail(c, GSPM_E_STATE, "mpnn_set_params before upload_mesh");
    hipSetDevice(c->device);
    int rc = nn_setup(c);
    if (rc) return static_cast<gspm_status>(rc);
    auto &nn = c->nn;
    hipStream_t s = c->stream;
    hipMemcpyAsync(nn.master, params, sizeof(float) * count, hipMemcpyHostToDevice, s);
    hipMemsetAsync(nn.m1, 0, sizeof(float) * count, s);
    hipMemsetAsync(nn.m2, 0, sizeof(float) * count, s);
    mpnn::launch_prepare_weights(nn.master, nn.wr, nn.mats, s);
    rc = hip_check(c, hipStreamSynchronize(s), "mpnn_set_params");
    if (rc) return static_cast<gspm_status>(rc);
    nn.adam_t = 0;
    nn.have_params = true;
    return GSPM_OK;
}

gspm_status gspm_mpnn_get_params(gspm_ctx *c, float *params, int64_t count) {
    if (!c) return GSPM_E_ARG;
    if (!params || count != mpnn::kNParam) return nfail(c, GSPM_E_ARG, "mpnn_get_params: need GSPM_MPNN_PARAMS floats");
    gspm_status st = nn_ready(c);
    if (st) return st;
    hipSetDevice(c->device);
    hipMemcpyAsync(params, c->nn.master, sizeof(float) * count, hipMemcpyDeviceToHost, c->stream);
    return static_cast<gspm_status>(hip_check(c, hipStreamSynchronize(c->stream), "mpnn_get_params"));
}

gspm_status gspm_mpnn_forward(gspm_ctx *c, const double *m_prev, const double *m, int64_t n_nodes, double *y,
                              double *s_m) {
    if (!c) return GSPM_E_ARG;
    if (!m_prev || !m || !y) return nfail(c, GSPM_E_ARG, "mpnn_forward: null array");
    gspm_status st = nn_ready(c);
    if (st) return st;
    if (n_nodes != c->n0) return nfail(c, GSPM_E_ARG, "mpnn_forward: n_nodes differs from the mesh");
    hipSetDevice(c->device);
    auto &nn = c->nn;
    int rc = upload_user(c, m_prev, nn.mp_in);
    rc = rc ? rc : upload_user(c, m, nn.m_in);
    if (rc) return static_cast<gspm_status>(rc);
    mpnn::launch_forward(nn.graph, c->mv, nn.net, nn.m_in, nn.mp_in, nn.red, nn.A, c->mat.l100, nullptr, c->stream);
    const size_t n = static_cast<size_t>(c->n);
    std::vector<float> yh(3 * n);
    std::vector<double> red(2 * kShards);
    hipMemcpyAsync(yh.data(), nn.y, sizeof(float) * 3 * n, hipMemcpyDeviceToHost, c->stream);
    hipMemcpyAsync(red.data(), nn.red, sizeof(double) * 2 * kShards, hipMemcpyDeviceToHost, c->stream);
    rc = hip_check(c, hipStreamSynchronize(c->stream), "mpnn_forward");
    if (rc) return static_cast<gspm_status>(rc);
    for (int64_t i = 0; i < c->n0; ++i) {
        const size_t k = static_cast<size_t>(c->user2int[i]);
        for (int a = 0; a < 3; ++a) y[3 * i + a] = yh[3 * k + a];
    }
    if (s_m) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < kShards; ++q) {
            a += red[q];
            b += red[kShards + q];
        }
        *s_m = b > 0.0 ? std::sqrt(a / b) : 0.0;
    }
    return GSPM_OK;
}

gspm_status gspm_mpnn_train_step(gspm_ctx *c, const double *m_prev, const double *m, const double *du,
                                 int64_t n_nodes, float lr, int32_t update, double *loss, float *grad) {
    if (!c) return GSPM_E_ARG;
    if (!m_prev || !m || !du) return nfail(c, GSPM_E_ARG, "mpnn_train_step: null array");
    if (!std::isfinite(lr) || lr < 0.0f) return nfail(c, GSPM_E_ARG, "mpnn_train_step: bad learning rate");
    gspm_status st = nn_ready(c);
    if (st) return st;
    if (!c->have_params) return nfail(c, GSPM_E_STATE, "mpnn_train_step needs set_params (lambda100)");
    if (n_nodes != c->n0) return nfail(c, GSPM_E_ARG, "mpnn_train_step: n_nodes differs from the mesh");
    hipSetDevice(c->device);
    auto &nn = c->nn;
    int rc = upload_user(c, m_prev, nn.mp_in);
    rc = rc ? rc : upload_user(c, m, nn.m_in);
    rc = rc ? rc : upload_user(c, du, nn.du);
    if (rc) return static_cast<gspm_status>(rc);
    hipStream_t s = c->stream;
    mpnn::launch_forward(nn.graph, c->mv, nn.net, nn.m_in, nn.mp_in, nn.red, nn.A, c->mat.l100, nullptr, s);
    mpnn::launch_loss_backward(nn.graph, c->mv, nn.net, nn.m_in, nn.mp_in, nn.du, c->mat.l100, nn.red, nn.A, nn.G,
                               nn.grad, s);
    if (grad) hipMemcpyAsync(grad, nn.grad, sizeof(float) * mpnn::kNParam, hipMemcpyDeviceToHost, s);
    if (update) {
        ++nn.adam_t;
        mpnn::launch_adam(nn.master, nn.grad, nn.m1, nn.m2, lr, nn.adam_t, s);
        mpnn::launch_prepare_weights(nn.master, nn.wr, nn.mats, s);
    }
    double red[kShards];
    hipMemcpyAsync(red, nn.red + mpnn::R_LOSS * kShards, sizeof red, hipMemcpyDeviceToHost, s);
    rc = hip_check(c, hipStreamSynchronize(s), "mpnn_train_step");
    if (rc) return static_cast<gspm_status>(rc);
    if (loss) {
        double a = 0.0;
        for (int q = 0; q < kShards; ++q) a += red[q];
        *loss = a;
    }
    return GSPM_OK;
}

gspm_status gspm_mpnn_warm_start(gspm_ctx *c, const double *m_prev, const double *u_prev, int64_t n_nodes, double *u0,
                                 double coef[2]) {
    if (!c) return GSPM_E_ARG;
    if (!m_prev || !u0) return nfail(c, GSPM_E_ARG, "mpnn_warm_start: null array");
    gspm_status st = nn_ready(c);
    if (st) return st;
    if (!c->have_params || !c->have_m) return nfail(c, GSPM_E_STATE, "mpnn_warm_start needs set_params and M");
    if (n_nodes != c->n0) return nfail(c, GSPM_E_ARG, "mpnn_warm_start: n_nodes differs from the mesh");
    hipSetDevice(c->device);
    auto &nn = c->nn;
    auto &d = c->d;
    int rc = upload_user(c, m_prev, nn.mp_in);
    if (!rc && u_prev) rc = upload_user(c, u_prev, nn.du);
    if (rc) return static_cast<gspm_status>(rc);
    hipStream_t s = c->stream;
    const size_t bytes3 = sizeof(double) * 3 * static_cast<size_t>(c->n);
    // the elastic right-hand side at the current m, as the step forms it
    launch_avg_sums(c->n, d.w, d.m, c->mat, d.sums, s, c->mv.det);
    launch_derive(d.sums, c->dargs, &d.der[0], s);
    hipMemcpyAsync(d.unext, d.u, bytes3, hipMemcpyDeviceToDevice, s);
    cg_prepare(c, 1);
    launch_elastic_rhs(c->mv, c->mat, d.m, d.b, d.unext, c->cg.bb, s);
    if (u_prev) {
        // the pinned node's displacement is zero in the start; so in u_prev
        std::vector<double> z(3, 0.0);
        for (int a = 0; a < 3; ++a)
            hipMemcpyAsync(nn.du + static_cast<size_t>(a) * c->n + c->p0, z.data(), sizeof(double),
                           hipMemcpyHostToDevice, s);
    }
    minres_start(c, d.m, nn.mp_in, u_prev ? nn.du : nullptr, d.unext, d.b);
    std::vector<double> h(3 * static_cast<size_t>(c->n));
    double ch[2] = {0.0, 0.0};
    hipMemcpyAsync(h.data(), d.unext, bytes3, hipMemcpyDeviceToHost, s);
    hipMemcpyAsync(ch, d.wcoef, sizeof ch, hipMemcpyDeviceToHost, s);
    rc = hip_check(c, hipStreamSynchronize(s), "mpnn_warm_start");
    if (rc) return static_cast<gspm_status>(rc);
    scatter_user(c, h, u0);
    if (coef) {
        coef[0] = ch[0];
        coef[1] = ch[1];
    }
    return GSPM_OK;
}

}  // extern "C"
