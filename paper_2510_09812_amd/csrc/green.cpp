// Host setup of the elastic preconditioner B = Q A_g^+ Q^T + omega D^-1
// (elastic_precond): the auxiliary grid, the restriction lists of Q^T, the
// diagonal of K^mech, the stencil of the grid operator (its symbol is
// inverted on the device), and the batched FFT plans.  The paper solves the
// elastic system by unpreconditioned CG and names that solve as the cost to
// cut (Sec. 5.2); the stiffness is one homogeneous C on a periodic cell, so
// the Green's operator of C on a regular periodic grid is close to its
// inverse.  The FFTs are plain library transforms (rocFFT); every other pass
// is a kernel of green_kernels.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include <rocfft/rocfft.h>

#include "context.h"

namespace gspm {

namespace {

constexpr double kOmega = 0.5;    // weight of the diagonal term

std::once_flag g_rocfft_once;
rocfft_status g_rocfft_setup = rocfft_status_success;

int fft_fail(gspm_ctx *c, const char *what) {
    c->err = std::string("elastic preconditioner: ") + what;
    return GSPM_E_DEVICE;
}

template <class T>
int pc_alloc(gspm_ctx *c, T **p, size_t count) {
    void *v = nullptr;
    const int rc = ctx_malloc(c, &v, sizeof(T) * std::max<size_t>(count, 1), "device allocation (elastic preconditioner)");
    *p = static_cast<T *>(v);
    return rc;
}

// Engineering strain (xx yy zz yz xz xy) of the displacement e_a phi for a
// basis function of gradient g.
void strain_of(int a, const double g[3], double e[6]) {
    for (int t = 0; t < 6; ++t) e[t] = 0.0;
    e[a] = g[a];
    if (a == 0) { e[4] = g[2]; e[5] = g[1]; }
    if (a == 1) { e[3] = g[2]; e[5] = g[0]; }
    if (a == 2) { e[3] = g[1]; e[4] = g[0]; }
}

double voigt_energy(const double C6[36], const double e[6], const double f[6]) {
    double v = 0.0;
    for (int r = 0; r < 6; ++r) {
        double row = 0.0;
        for (int q = 0; q < 6; ++q) row += C6[6 * r + q] * f[q];
        v += e[r] * row;
    }
    return v;
}

// Barycentric gradients of a tetrahedron from its three edge vectors (rows);
// returns the volume.
double edge_grads(const double E[3][3], double g[4][3]) {
    double c[3][3];
    for (int k = 0; k < 3; ++k) {
        const double *a = E[(k + 1) % 3], *b = E[(k + 2) % 3];
        c[k][0] = a[1] * b[2] - a[2] * b[1];
        c[k][1] = a[2] * b[0] - a[0] * b[2];
        c[k][2] = a[0] * b[1] - a[1] * b[0];
    }
    const double det = E[0][0] * c[0][0] + E[0][1] * c[0][1] + E[0][2] * c[0][2];
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 3; ++a) g[k + 1][a] = c[k][a] / det;
    for (int a = 0; a < 3; ++a) g[0][a] = -(g[1][a] + g[2][a] + g[3][a]);
    return std::fabs(det) / 6.0;
}

// 3x3 blocks S(o) coupling a grid node to the node at offset o, from the six
// tetrahedra of a cell split around its main diagonal.
void grid_stencil(const double C6[36], const double h[3], double S[27 * 9]) {
    std::memset(S, 0, sizeof(double) * 27 * 9);
    const int order[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (const auto &ord : order) {
        int off[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int v = 1; v < 4; ++v) {
            for (int a = 0; a < 3; ++a) off[v][a] = off[v - 1][a];
            off[v][ord[v - 1]] += 1;
        }
        double E[3][3], g[4][3];
        for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 3; ++a) E[k][a] = (off[k + 1][a] - off[0][a]) * h[a];
        const double V = edge_grads(E, g);
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                const int ox = off[j][0] - off[i][0], oy = off[j][1] - off[i][1], oz = off[j][2] - off[i][2];
                double *blk = S + 9 * ((oz + 1) * 9 + (oy + 1) * 3 + (ox + 1));
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        double ea[6], eb[6];
                        strain_of(a, g[i], ea);
                        strain_of(b, g[j], eb);
                        blk[3 * a + b] += V * voigt_energy(C6, ea, eb);
                    }
            }
    }
}

int make_plans(gspm_ctx *c, bool f32) {
    std::call_once(g_rocfft_once, []() { g_rocfft_setup = rocfft_setup(); });
    if (g_rocfft_setup != rocfft_status_success) return fft_fail(c, "rocfft_setup failed");
    auto &pc = c->pc;
    const size_t len[3] = {static_cast<size_t>(pc.gv.gx), static_cast<size_t>(pc.gv.gy),
                           static_cast<size_t>(pc.gv.gz)};
    const rocfft_precision prec = f32 ? rocfft_precision_single : rocfft_precision_double;
    // the three real fields packed into two complex ones, transformed as one batch (grid -> spec, spec -> grid)
    rocfft_plan fwd = nullptr, inv = nullptr;
    if (rocfft_plan_create(&fwd, rocfft_placement_notinplace, rocfft_transform_type_complex_forward, prec, 3, len, 2,
                           nullptr) != rocfft_status_success)
        return fft_fail(c, "rocfft_plan_create (forward) failed");
    pc.fwd = fwd;
    if (rocfft_plan_create(&inv, rocfft_placement_notinplace, rocfft_transform_type_complex_inverse, prec, 3, len, 2,
                           nullptr) != rocfft_status_success)
        return fft_fail(c, "rocfft_plan_create (inverse) failed");
    pc.inv = inv;
    size_t w1 = 0, w2 = 0;
    rocfft_plan_get_work_buffer_size(fwd, &w1);
    rocfft_plan_get_work_buffer_size(inv, &w2);
    pc.work_bytes = std::max(w1, w2);
    if (pc.work_bytes) {
        int rc = pc_alloc(c, reinterpret_cast<char **>(&pc.work), pc.work_bytes);
        if (rc) return rc;
    }
    rocfft_execution_info info = nullptr;
    if (rocfft_execution_info_create(&info) != rocfft_status_success) return fft_fail(c, "execution info");
    pc.info = info;
    if (rocfft_execution_info_set_stream(info, c->stream) != rocfft_status_success) return fft_fail(c, "set stream");
    if (pc.work_bytes &&
        rocfft_execution_info_set_work_buffer(info, pc.work, pc.work_bytes) != rocfft_status_success)
        return fft_fail(c, "set work buffer");
    return GSPM_OK;
}

// The grid and the restriction lists: grid point g gathers every node whose
// trilinear corners include g, with that corner's weight.
int setup_mesh_part(gspm_ctx *c) {
    auto &pc = c->pc;
    auto &gv = pc.gv;
    const int n = c->n;
    const bool f32 = c->precision == GSPM_MIXED;
    const double ell = std::cbrt(c->vc / n);
    const double L[3] = {c->mv.Lx, c->mv.Ly, c->mv.Lz};
    int g[3];
    for (int a = 0; a < 3; ++a) {
        g[a] = std::max(2, static_cast<int>(std::floor(L[a] / ell + 0.5)));
        gv.h[a] = L[a] / g[a];
    }
    gv.gx = g[0]; gv.gy = g[1]; gv.gz = g[2];
    gv.gxh = g[0] / 2 + 1;
    gv.G = static_cast<int64_t>(g[0]) * g[1] * g[2];
    gv.Gh = static_cast<int64_t>(gv.gxh) * g[1] * g[2];
    if (gv.G > (int64_t{1} << 30)) {
        c->err = "elastic preconditioner: grid too large";
        return GSPM_E_ARG;
    }
    for (int a = 0; a < 3; ++a) gv.lo[a] = c->box_lo[a];
    std::vector<double> xs(3 * static_cast<size_t>(n));
    int rc = hip_check(c, hipMemcpyAsync(xs.data(), c->d.x, sizeof(double) * xs.size(), hipMemcpyDeviceToHost,
                                         c->stream), "elastic preconditioner setup");
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "elastic preconditioner setup");
    if (rc) return rc;
    // the eight (grid point, weight) pairs of every node, as k_pc_prolong forms them
    std::vector<int64_t> gidx(8 * static_cast<size_t>(n));
    std::vector<double> wts(8 * static_cast<size_t>(n));
    for (int i = 0; i < n; ++i) {
        int i0[3], i1[3];
        double t[3];
        for (int a = 0; a < 3; ++a) {
            double f = (xs[static_cast<size_t>(a) * n + i] - gv.lo[a]) / gv.h[a];
            f -= g[a] * std::floor(f / g[a]);
            int k = static_cast<int>(std::floor(f));
            if (k >= g[a]) k = g[a] - 1;
            if (k < 0) k = 0;
            i0[a] = k;
            i1[a] = k + 1 == g[a] ? 0 : k + 1;
            t[a] = f - k;
        }
        for (int cc = 0; cc < 8; ++cc) {
            const int ix = (cc & 1) ? i1[0] : i0[0], iy = (cc & 2) ? i1[1] : i0[1], iz = (cc & 4) ? i1[2] : i0[2];
            gidx[8 * static_cast<size_t>(i) + cc] = (static_cast<int64_t>(iz) * g[1] + iy) * g[0] + ix;
            wts[8 * static_cast<size_t>(i) + cc] = ((cc & 1) ? t[0] : 1.0 - t[0]) * ((cc & 2) ? t[1] : 1.0 - t[1]) *
                                                   ((cc & 4) ? t[2] : 1.0 - t[2]);
        }
    }
    // rows of the restriction run over the grid points in Morton order (the
    // nodes are Morton-numbered, so consecutive rows gather nearby nodes)
    auto spread = [](uint64_t v) {
        uint64_t x = v & 0x1FFFFFu;
        x = (x | (x << 32)) & 0x1F00000000FFFFull;
        x = (x | (x << 16)) & 0x1F0000FF0000FFull;
        x = (x | (x << 8)) & 0x100F00F00F00F00Full;
        x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
        x = (x | (x << 2)) & 0x1249249249249249ull;
        return x;
    };
    std::vector<std::pair<uint64_t, int32_t>> order(static_cast<size_t>(gv.G));
    for (int64_t q = 0; q < gv.G; ++q) {
        const uint64_t ix = q % g[0], iy = (q / g[0]) % g[1], iz = q / (static_cast<int64_t>(g[0]) * g[1]);
        order[q] = {spread(ix) | (spread(iy) << 1) | (spread(iz) << 2), static_cast<int32_t>(q)};
    }
    std::sort(order.begin(), order.end());
    std::vector<int32_t> row_of(static_cast<size_t>(gv.G)), rgrid(static_cast<size_t>(gv.G));
    for (int64_t t = 0; t < gv.G; ++t) {
        rgrid[t] = order[t].second;
        row_of[static_cast<size_t>(order[t].second)] = static_cast<int32_t>(t);
    }
    std::vector<int32_t> ptr(static_cast<size_t>(gv.G) + 1, 0), node(8 * static_cast<size_t>(n));
    for (int64_t q : gidx) ++ptr[static_cast<size_t>(row_of[static_cast<size_t>(q)]) + 1];
    for (int64_t q = 0; q < gv.G; ++q) ptr[q + 1] += ptr[q];
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    std::vector<double> w64(8 * static_cast<size_t>(n));
    for (int i = 0; i < n; ++i)      // nodes in order within each list
        for (int cc = 0; cc < 8; ++cc) {
            const size_t e = 8 * static_cast<size_t>(i) + cc;
            const int32_t slot = fill[static_cast<size_t>(row_of[static_cast<size_t>(gidx[e])])]++;
            node[slot] = i;
            w64[slot] = wts[e];
        }
    const size_t tb = f32 ? sizeof(float) : sizeof(double);
    rc = pc_alloc(c, &pc.rptr, ptr.size());
    if (!rc) rc = pc_alloc(c, &pc.rgrid, rgrid.size());
    if (!rc) rc = pc_alloc(c, &pc.rnode, node.size());
    if (!rc) rc = pc_alloc(c, reinterpret_cast<char **>(&pc.rw), tb * w64.size());
    if (!rc) rc = pc_alloc(c, reinterpret_cast<char **>(&pc.dinv), tb * 3 * static_cast<size_t>(n));
    if (!rc) rc = pc_alloc(c, reinterpret_cast<char **>(&pc.ainv), tb * 9 * static_cast<size_t>(gv.Gh));
    if (!rc) rc = pc_alloc(c, reinterpret_cast<char **>(&pc.grid), tb * 4 * static_cast<size_t>(gv.G));
    if (!rc) rc = pc_alloc(c, reinterpret_cast<char **>(&pc.spec), tb * 4 * static_cast<size_t>(gv.G));
    if (!rc) rc = pc_alloc(c, &pc.aux, 3 * kShards + 3);
    if (rc) return rc;
    hipMemcpyAsync(pc.rptr, ptr.data(), sizeof(int32_t) * ptr.size(), hipMemcpyHostToDevice, c->stream);
    hipMemcpyAsync(pc.rnode, node.data(), sizeof(int32_t) * node.size(), hipMemcpyHostToDevice, c->stream);
    hipMemcpyAsync(pc.rgrid, rgrid.data(), sizeof(int32_t) * rgrid.size(), hipMemcpyHostToDevice, c->stream);
    if (f32) {
        std::vector<float> w32(w64.begin(), w64.end());
        hipMemcpyAsync(pc.rw, w32.data(), sizeof(float) * w32.size(), hipMemcpyHostToDevice, c->stream);
        rc = hip_check(c, hipStreamSynchronize(c->stream), "elastic preconditioner setup");
    } else {
        hipMemcpyAsync(pc.rw, w64.data(), sizeof(double) * w64.size(), hipMemcpyHostToDevice, c->stream);
        rc = hip_check(c, hipStreamSynchronize(c->stream), "elastic preconditioner setup");
    }
    if (rc) return rc;
    gv.rptr = pc.rptr;
    gv.rgrid = pc.rgrid;
    gv.rnode = pc.rnode;
    gv.rw = pc.rw;
    gv.dinv = pc.dinv;
    gv.ainv = pc.ainv;
    gv.grid = pc.grid;
    gv.spec = pc.spec;
    rc = make_plans(c, f32);
    if (rc) return rc;
    pc.mesh_ready = true;
    return GSPM_OK;
}

// omega / diag(K^mech) at every node (all elements, nearest-image edges).
int setup_diagonal(gspm_ctx *c, double factor, bool f32) {
    const int n = c->n;
    std::vector<double> xs(3 * static_cast<size_t>(n));
    int rc = hip_check(c, hipMemcpyAsync(xs.data(), c->d.x, sizeof(double) * xs.size(), hipMemcpyDeviceToHost,
                                         c->stream), "elastic preconditioner setup");
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "elastic preconditioner setup");
    if (rc) return rc;
    const double L[3] = {c->mv.Lx, c->mv.Ly, c->mv.Lz};
    std::vector<double> diag(3 * static_cast<size_t>(n), 0.0);
    const int64_t ne = c->ne;
    for (int64_t e = 0; e < ne; ++e) {
        const int32_t *v = &c->tets_int[4 * static_cast<size_t>(e)];
        double E[3][3], g[4][3];
        for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 3; ++a) {
                double d = xs[static_cast<size_t>(a) * n + v[k + 1]] - xs[static_cast<size_t>(a) * n + v[0]];
                d -= L[a] * std::nearbyint(d / L[a]);
                E[k][a] = d;
            }
        const double V = edge_grads(E, g);
        for (int j = 0; j < 4; ++j)
            for (int a = 0; a < 3; ++a) {
                double ea[6];
                strain_of(a, g[j], ea);
                diag[static_cast<size_t>(a) * n + v[j]] += V * voigt_energy(c->mat.C6, ea, ea);
            }
    }
    std::vector<double> dinv(diag.size());
    for (size_t i = 0; i < diag.size(); ++i) dinv[i] = kOmega * factor / diag[i];
    if (f32) {
        std::vector<float> d32(dinv.begin(), dinv.end());
        hipMemcpyAsync(c->pc.dinv, d32.data(), sizeof(float) * d32.size(), hipMemcpyHostToDevice, c->stream);
        return hip_check(c, hipStreamSynchronize(c->stream), "elastic preconditioner setup");
    }
    hipMemcpyAsync(c->pc.dinv, dinv.data(), sizeof(double) * dinv.size(), hipMemcpyHostToDevice, c->stream);
    return hip_check(c, hipStreamSynchronize(c->stream), "elastic preconditioner setup");
}

}  // namespace

int green_setup(gspm_ctx *c) {
    auto &pc = c->pc;
    if (!pc.mesh_ready) {
        const int rc = setup_mesh_part(c);
        if (rc) {
            c->release_pc();
            return rc;
        }
    }
    // the mixed form's FP32 inner solves run A' = A / (len_scale c11): their
    // preconditioner carries the inverse factor
    const bool f32 = c->precision == GSPM_MIXED;
    const double factor = f32 ? c->mv.len_scale * c->mat.c11 : 1.0;
    double key[37];
    std::memcpy(key, c->mat.C6, sizeof(double) * 36);
    key[36] = factor;
    if (pc.sym_ready && std::memcmp(key, pc.sym_key, sizeof key) == 0) return GSPM_OK;
    pc.sym_ready = false;
    double S[27 * 9];
    grid_stencil(c->mat.C6, pc.gv.h, S);
    if (f32)
        launch_pc_symbol<float>(pc.gv, S, factor / static_cast<double>(pc.gv.G), c->stream);
    else
        launch_pc_symbol<double>(pc.gv, S, factor / static_cast<double>(pc.gv.G), c->stream);
    int rc = setup_diagonal(c, factor, f32);
    if (rc) return rc;
    std::memcpy(pc.sym_key, key, sizeof key);
    pc.sym_ready = true;
    return GSPM_OK;
}

int green_fft(gspm_ctx *c, bool forward) {
    auto &pc = c->pc;
    void *in[1] = {forward ? pc.grid : pc.spec};
    void *out[1] = {forward ? pc.spec : pc.grid};
    const rocfft_status st = rocfft_execute(static_cast<rocfft_plan>(forward ? pc.fwd : pc.inv), in, out,
                                            static_cast<rocfft_execution_info>(pc.info));
    return st == rocfft_status_success ? GSPM_OK : fft_fail(c, "rocfft_execute failed");
}

int green_apply64(gspm_ctx *c, const double *x, double *y) {
    auto &pc = c->pc;
    // a fresh scalar set: the passes test nothing (test_k < 0) and run
    cg_prepare(c, 1);
    launch_pc_restrict<double>(pc.gv, c->n, x, c->cg, -1, 0.0, c->stream);
    int rc = green_fft(c, true);
    if (rc) return rc;
    launch_pc_modes<double>(pc.gv, c->cg, c->stream);
    rc = green_fft(c, false);
    if (rc) return rc;
    launch_pc_prolong<double>(pc.gv, c->mv, x, y, c->cg.rq_at(0), c->cg, c->stream);
    return hip_check(c, hipStreamSynchronize(c->stream), "apply(PRECOND)");
}

}  // namespace gspm

void gspm_ctx::release_pc() {
    if (stream) hipStreamSynchronize(stream);
    auto &q = pc;
    if (q.fwd) rocfft_plan_destroy(static_cast<rocfft_plan>(q.fwd));
    if (q.inv) rocfft_plan_destroy(static_cast<rocfft_plan>(q.inv));
    if (q.info) rocfft_execution_info_destroy(static_cast<rocfft_execution_info>(q.info));
    for (void *p : {static_cast<void *>(q.rptr), static_cast<void *>(q.rgrid), static_cast<void *>(q.rnode), q.rw,
                    q.dinv, q.ainv, q.grid, q.spec, q.work, static_cast<void *>(q.aux)})
        gspm::ctx_free(this, p);
    q = gspm::GreenState{};
}
