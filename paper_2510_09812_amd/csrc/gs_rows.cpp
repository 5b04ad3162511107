// Host assembly of the GS operator's rows (upload time).
//
// The GS solves (Alg. B.1) apply eps K + M over the magnetic elements, with
// the P1 element matrices of Sec. 2.3: K^e_ij = V g_i . g_j and
// M^e_ij = V (1 + delta_ij) / 20.  Both parts share one sparsity pattern (the
// node's edge neighbours through magnetic elements), so the operator is
// stored once per mesh as its two coefficient sets and applied row by row:
// per node about 14 coefficients and 14 column indices instead of the
// geometry of its ~24 elements, recomputed by every block that touches them.
//
// Layout: rows in the library's node order, grouped in slices of 64 (one
// wavefront, one lane per row).  A slice stores its rows' off-diagonal
// entries entry-major: entry k of lane l at off[s] + 64 k + l, padded to the
// slice's longest row with zero coefficients that point at the row itself.
// Columns are 16-bit indices into the row's block staging: the block's owned
// range, then its sorted halo list, which holds exactly the columns outside
// the range.  Row blocks are ranges of the node order like the element
// blocks, of a size of their own: the row kernels carry less per node than
// the element kernels, so larger blocks amortise their per-block work and
// stage fewer halo nodes per owned node.  The diagonal is kept apart.
#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <thread>

#include "common.h"

namespace gspm {

namespace {

// Gradients of the barycentric coordinates and the volume of element e (its
// vertices as internal node ids), edges taken to the nearest periodic image.
void element_gradients(const HostMesh &hm, const int32_t (&v)[4], double (&g)[4][3], double &V) {
    const size_t n = static_cast<size_t>(hm.n);
    double E[3][3];
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 3; ++a) {
            double d = hm.xs[a * n + static_cast<size_t>(v[k + 1])] - hm.xs[a * n + static_cast<size_t>(v[0])];
            d -= hm.L[a] * std::nearbyint(d / hm.L[a]);
            E[k][a] = d;
        }
    double cf[3][3];
    for (int k = 0; k < 3; ++k) {
        const double *p = E[(k + 1) % 3], *q = E[(k + 2) % 3];
        cf[k][0] = p[1] * q[2] - p[2] * q[1];
        cf[k][1] = p[2] * q[0] - p[0] * q[2];
        cf[k][2] = p[0] * q[1] - p[1] * q[0];
    }
    const double det = E[0][0] * cf[0][0] + E[0][1] * cf[0][1] + E[0][2] * cf[0][2];
    V = std::fabs(det) / 6.0;
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 3; ++a) g[k + 1][a] = cf[k][a] / det;
    for (int a = 0; a < 3; ++a) g[0][a] = -(g[1][a] + g[2][a] + g[3][a]);
}

// Runs body(i) for every i in [0, n) on the host's threads, in chunks.
template <class Body>
void for_rows(int32_t n, Body body, int32_t kChunk = 2048) {
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::atomic<int32_t> next{0};
    auto worker = [&]() {
        for (;;) {
            const int32_t i0 = next.fetch_add(kChunk);
            if (i0 >= n) return;
            const int32_t i1 = std::min(n, i0 + kChunk);
            for (int32_t i = i0; i < i1; ++i) body(i);
        }
    };
    std::vector<std::thread> pool;
    for (unsigned t = 1; t < hw; ++t) pool.emplace_back(worker);
    worker();
    for (auto &t : pool) t.join();
}

}  // namespace

int assemble_gs_rows(const HostMesh &hm, int64_t ne, const int32_t *tets, const uint8_t *tags, int32_t nb_rows,
                     GsRowsHost &out, std::string &err) {
    const int32_t n = hm.n, nb = nb_rows > 0 ? nb_rows : hm.nb;
    if (nb % 64 != 0) {
        err = "GS rows: blocks must hold a multiple of 64 nodes";
        return GSPM_E_ARG;
    }
    // incidence of the magnetic elements, in element order
    std::vector<int64_t> iptr(static_cast<size_t>(n) + 1, 0);
    for (int64_t e = 0; e < ne; ++e)
        if (tags[e])
            for (int j = 0; j < 4; ++j) ++iptr[static_cast<size_t>(hm.user2int[tets[4 * e + j]]) + 1];
    for (int32_t i = 0; i < n; ++i) iptr[i + 1] += iptr[i];
    std::vector<int32_t> inc(static_cast<size_t>(iptr[n]));
    {
        std::vector<int64_t> cur(iptr.begin(), iptr.end() - 1);
        for (int64_t e = 0; e < ne; ++e)
            if (tags[e])
                for (int j = 0; j < 4; ++j) inc[cur[hm.user2int[tets[4 * e + j]]]++] = static_cast<int32_t>(e);
    }
    auto vertices = [&](int32_t e, int32_t (&v)[4]) {
        for (int j = 0; j < 4; ++j) v[j] = hm.user2int[tets[4 * static_cast<int64_t>(e) + j]];
    };
    // pass 1: the distinct neighbours of each row
    std::vector<int64_t> rptr(static_cast<size_t>(n) + 1, 0);
    for_rows(n, [&](int32_t i) {
        int32_t nbr[256];
        int cnt = 0;
        for (int64_t t = iptr[i]; t < iptr[i + 1]; ++t) {
            int32_t v[4];
            vertices(inc[t], v);
            for (int j = 0; j < 4; ++j) {
                if (v[j] == i) continue;
                bool seen = false;
                for (int q = 0; q < cnt && !seen; ++q) seen = nbr[q] == v[j];
                if (!seen && cnt < 256) nbr[cnt++] = v[j];
            }
        }
        rptr[i + 1] = cnt;
    });
    for (int32_t i = 0; i < n; ++i) {
        if (rptr[i + 1] >= 256) {
            err = "GS rows: a node has 256 or more neighbours";
            return GSPM_E_MESH;
        }
        rptr[i + 1] += rptr[i];
    }
    // pass 2: the coefficients, summed over the row's elements in incidence order
    std::vector<int32_t> ccol(static_cast<size_t>(rptr[n]));
    std::vector<double> ck(ccol.size(), 0.0), cm(ccol.size(), 0.0);
    out.kd.assign(n, 0.0);
    out.md.assign(n, 0.0);
    for_rows(n, [&](int32_t i) {
        const int64_t r0 = rptr[i];
        int cnt = 0;
        for (int64_t t = iptr[i]; t < iptr[i + 1]; ++t) {
            int32_t v[4];
            vertices(inc[t], v);
            double g[4][3], V;
            element_gradients(hm, v, g, V);
            int a = 0;
            while (v[a] != i) ++a;
            for (int b = 0; b < 4; ++b) {
                const double kab = V * (g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2]);
                if (v[b] == i) {
                    out.kd[i] += kab;
                    out.md[i] += b == a ? V / 10.0 : V / 20.0;
                    continue;
                }
                int q = 0;
                while (q < cnt && ccol[r0 + q] != v[b]) ++q;
                if (q == cnt) ccol[r0 + cnt++] = v[b];
                ck[r0 + q] += kab;
                cm[r0 + q] += V / 20.0;
            }
        }
        // columns in ascending node order (coefficients follow)
        std::vector<int> ord(cnt);
        for (int q = 0; q < cnt; ++q) ord[q] = q;
        std::sort(ord.begin(), ord.end(), [&](int x, int y) { return ccol[r0 + x] < ccol[r0 + y]; });
        int32_t c2[256];
        double k2[256], m2[256];
        for (int q = 0; q < cnt; ++q) {
            c2[q] = ccol[r0 + ord[q]];
            k2[q] = ck[r0 + ord[q]];
            m2[q] = cm[r0 + ord[q]];
        }
        for (int q = 0; q < cnt; ++q) {
            ccol[r0 + q] = c2[q];
            ck[r0 + q] = k2[q];
            cm[r0 + q] = m2[q];
        }
    });
    // row blocks: the halo of a block is the set of its rows' columns outside its owned range
    out.nb = nb;
    out.nblk = (n + nb - 1) / nb;
    std::vector<std::vector<int32_t>> halos(static_cast<size_t>(out.nblk));
    for_rows(out.nblk, [&](int32_t b) {
        const int32_t n0 = b * nb, n1 = std::min(n, n0 + nb);
        auto &h = halos[b];
        for (int64_t t = rptr[n0]; t < rptr[n1]; ++t)
            if (ccol[t] < n0 || ccol[t] >= n1) h.push_back(ccol[t]);
        std::sort(h.begin(), h.end());
        h.erase(std::unique(h.begin(), h.end()), h.end());
    }, 8);
    out.halo_ptr.assign(static_cast<size_t>(out.nblk) + 1, 0);
    out.nloc_max = 0;
    for (int32_t b = 0; b < out.nblk; ++b) {
        const int64_t nloc = static_cast<int64_t>(nb) + static_cast<int64_t>(halos[b].size());
        if (nloc > 65535) {
            err = "GS rows: a row block stages more than 65535 nodes";
            return GSPM_E_MESH;
        }
        out.nloc_max = std::max(out.nloc_max, static_cast<int32_t>(nloc));
        out.halo_ptr[b + 1] = out.halo_ptr[b] + static_cast<int32_t>(halos[b].size());
    }
    out.halo_ids.resize(static_cast<size_t>(out.halo_ptr[out.nblk]));
    for (int32_t b = 0; b < out.nblk; ++b)
        std::copy(halos[b].begin(), halos[b].end(), out.halo_ids.begin() + out.halo_ptr[b]);
    // sliced rows with block-local columns
    const int32_t nsl = (n + 63) / 64;
    out.off.assign(static_cast<size_t>(nsl) + 1, 0);
    int64_t total = 0;
    for (int32_t s = 0; s < nsl; ++s) {
        int64_t w = 0;
        for (int32_t i = 64 * s; i < std::min(n, 64 * s + 64); ++i) w = std::max(w, rptr[i + 1] - rptr[i]);
        total += 64 * w;
        if (total > INT32_MAX) {
            err = "GS rows: more than 2^31 entries";
            return GSPM_E_MESH;
        }
        out.off[s + 1] = static_cast<int32_t>(total);
    }
    out.col.assign(static_cast<size_t>(out.off[nsl]), 0);
    out.kv.assign(out.col.size(), 0.0);
    out.mv.assign(out.col.size(), 0.0);
    std::atomic<int> bad{0};
    for_rows(n, [&](int32_t i) {
        const int32_t b = i / nb, n0 = b * nb, s = i / 64, lane = i % 64;
        const int32_t *h0 = out.halo_ids.data() + out.halo_ptr[b], *h1 = out.halo_ids.data() + out.halo_ptr[b + 1];
        const int64_t w = (out.off[s + 1] - out.off[s]) / 64, cnt = rptr[i + 1] - rptr[i];
        for (int64_t q = 0; q < w; ++q) {
            const size_t e = static_cast<size_t>(out.off[s]) + 64 * static_cast<size_t>(q) + lane;
            if (q >= cnt) {
                out.col[e] = static_cast<uint16_t>(i - n0);
                continue;
            }
            const int32_t j = ccol[rptr[i] + q];
            int32_t loc;
            if (j >= n0 && j < n0 + nb) {
                loc = j - n0;
            } else {
                const int32_t *it = std::lower_bound(h0, h1, j);
                if (it == h1 || *it != j) {
                    bad = 1;
                    return;
                }
                loc = nb + static_cast<int32_t>(it - h0);
            }
            out.col[e] = static_cast<uint16_t>(loc);
            out.kv[e] = ck[rptr[i] + q];
            out.mv[e] = cm[rptr[i] + q];
        }
    });
    if (bad) {
        err = "GS rows: a neighbour is missing from its block's staged nodes";
        return GSPM_E_MESH;
    }
    return GSPM_OK;
}

}  // namespace gspm
