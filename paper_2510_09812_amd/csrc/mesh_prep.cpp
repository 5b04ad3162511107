// One-time host preprocessing of an uploaded mesh.
//
//  1. Periodic identification (Sec. 2.5): every node on a max face of the box
//     is wrapped onto the min face; nodes whose wrapped coordinates agree (to
//     1e-9 of the box edge) are one unique node.  A hash table keyed by the
//     quantised coordinates of the min-face representatives does the matching.
//  2. Validation and geometry in FP64: repeated vertices, degenerate elements,
//     lumped magnetic weights w_j = sum_e chi_e V_e / 4 (the volume-average
//     weights of Sec. 2.4) and the cell volume.
//  3. Renumbering of the unique nodes along a Morton (Z-order) curve, so that
//     a contiguous range of node ids is a compact patch of the mesh.
//  4. Owner blocks: block b owns the node range [b*nb, (b+1)*nb) and lists
//     every element with a vertex in that range (magnetic elements first).
//     An element pass runs one workgroup per block, accumulates the
//     contributions to owned nodes in LDS, and writes each owned node once.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_map>

#include "common.h"

namespace gspm {

namespace {

struct KeyHash {
    size_t operator()(const std::array<int64_t, 3> &k) const noexcept {
        uint64_t h = 1469598103934665603ull;
        for (int a = 0; a < 3; ++a) {
            h ^= static_cast<uint64_t>(k[a]) + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
        }
        return static_cast<size_t>(h);
    }
};

uint64_t spread3(uint64_t v) {   // 21 bits -> every third bit of 63
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

}  // namespace

int nodes_per_block(int32_t requested, int64_t n) {
    if (requested > 0) return requested;
    (void)n;
    return 256;
}

// Orders one group of a block's elements (4 local vertex ids each) into
// strips of face-adjacent tetrahedra: a greedy walk that prefers the
// neighbour with the fewest unvisited neighbours.
static void strip_order(const uint16_t *lc, int32_t m, std::vector<int32_t> &order) {
    order.clear();
    if (m <= 0) return;
    std::vector<std::pair<uint64_t, int32_t>> faces;
    faces.reserve(4 * static_cast<size_t>(m));
    for (int32_t e = 0; e < m; ++e) {
        uint16_t v[4] = {lc[4 * e], lc[4 * e + 1], lc[4 * e + 2], lc[4 * e + 3]};
        std::sort(v, v + 4);
        for (int skip = 0; skip < 4; ++skip) {
            uint64_t key = 0;
            for (int j = 0; j < 4; ++j)
                if (j != skip) key = (key << 16) | v[j];
            faces.emplace_back(key, e);
        }
    }
    std::sort(faces.begin(), faces.end());
    std::vector<int32_t> adj(4 * static_cast<size_t>(m), -1);
    std::vector<int8_t> nadj(static_cast<size_t>(m), 0);
    for (size_t i = 0; i + 1 < faces.size(); ++i)
        if (faces[i].first == faces[i + 1].first) {
            const int32_t a = faces[i].second, c = faces[i + 1].second;
            if (nadj[a] < 4 && nadj[c] < 4) {
                adj[4 * a + nadj[a]++] = c;
                adj[4 * c + nadj[c]++] = a;
            }
        }
    std::vector<uint8_t> vis(static_cast<size_t>(m), 0);
    auto free_nbrs = [&](int32_t e) {
        int k = 0;
        for (int j = 0; j < nadj[e]; ++j) k += !vis[adj[4 * e + j]];
        return k;
    };
    order.reserve(static_cast<size_t>(m));
    for (int32_t s0 = 0; s0 < m; ++s0) {
        if (vis[s0]) continue;
        int32_t cur = s0;
        vis[cur] = 1;
        order.push_back(cur);
        for (;;) {
            int32_t best = -1, bestk = 5;
            for (int j = 0; j < nadj[cur]; ++j) {
                const int32_t c = adj[4 * cur + j];
                if (vis[c]) continue;
                const int k = free_nbrs(c);
                if (k < bestk) { bestk = k; best = c; }
            }
            if (best < 0) break;
            cur = best;
            vis[cur] = 1;
            order.push_back(cur);
        }
    }
}

// Packs a strip order into segments of at most `budget` window updates (an
// element's updates never straddle two segments).  Along a strip an element
// costs one vertex load; at a strip break the missing vertices are loaded
// first.  A segment opens with its first element's four vertices in slots
// 0..3, in order.  After that every load follows the kernels' rotation: the
// entering vertex takes slot 3 and the vertex held in slot 3 moves into the
// slot of the vertex that leaves, which is one the element does not use (the
// least recently used).  An entry names the leaving vertex's slot, so at a
// flagged entry the four slots hold exactly the element's vertices.  With
// `emit` false only the number of segments is returned.
static int32_t pack_strips(const uint16_t *lc, const std::vector<int32_t> &order, int budget, bool emit,
                           std::vector<uint16_t> &ent, std::vector<uint32_t> &off, std::vector<uint16_t> &nent) {
    int32_t win[4] = {-1, -1, -1, -1};
    int64_t lru[4] = {0, 0, 0, 0}, clock = 0;
    int used = 0;
    int32_t segs = 0;
    auto close = [&]() {
        if (emit) {
            nent.push_back(static_cast<uint16_t>(used));
            while (ent.size() % 8) ent.push_back(0);
        }
        for (int k = 0; k < 4; ++k) win[k] = -1;
        used = 0;
    };
    for (int32_t e : order) {
        const int32_t v[4] = {lc[4 * e], lc[4 * e + 1], lc[4 * e + 2], lc[4 * e + 3]};
        auto in_win = [&](int32_t x) { return x == win[0] || x == win[1] || x == win[2] || x == win[3]; };
        auto in_elem = [&](int32_t x) { return x == v[0] || x == v[1] || x == v[2] || x == v[3]; };
        int nnew = 0;
        for (int j = 0; j < 4; ++j) nnew += !in_win(v[j]);
        if (used > 0 && used + nnew > budget) close();
        if (used == 0) {
            // the opening element: its vertices straight into slots 0..3
            ++segs;
            if (emit) off.push_back(static_cast<uint32_t>(ent.size() / 8));
            for (int j = 0; j < 4; ++j) {
                win[j] = v[j];
                if (emit) ent.push_back(static_cast<uint16_t>(v[j] | (j << 14) | (j == 3 ? kEntElem : 0u)));
            }
            used = 4;
        } else {
            for (int j = 0; j < 4; ++j) {
                if (in_win(v[j])) continue;
                int slot = -1;
                for (int k = 0; k < 4; ++k) {
                    if (in_elem(win[k])) continue;      // the element still needs this vertex
                    if (slot < 0 || lru[k] < lru[slot]) slot = k;
                }
                win[slot] = win[3];                     // slot 3's vertex moves into the freed slot
                lru[slot] = lru[3];
                win[3] = v[j];                          // the entering vertex takes slot 3
                lru[3] = 0;
                ++used;
                if (emit) ent.push_back(static_cast<uint16_t>(v[j] | (slot << 14)));
            }
            if (emit) ent.back() = static_cast<uint16_t>(ent.back() | kEntElem);
        }
        for (int k = 0; k < 4; ++k)
            if (in_elem(win[k])) lru[k] = ++clock;
    }
    if (used > 0) close();
    return segs;
}

int prepare_mesh(int64_t n0, const double *xyz, int64_t ne, const int32_t *tets, const uint8_t *tags,
                 const double lo[3], const double hi[3], int32_t nb, HostMesh &M, std::string &err, int reorder) {
    M = HostMesh();
    if (n0 < 4 || ne < 1 || n0 > INT32_MAX || ne > INT32_MAX) { err = "mesh needs 4..2^31-1 nodes and >= 1 tetrahedron"; return GSPM_E_ARG; }
    if (nb < 64 || nb > 1024 || (nb & (nb - 1))) { err = "block_nodes must be a power of two in [64, 1024]"; return GSPM_E_ARG; }
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(lo[a]) || !std::isfinite(hi[a]) || !(hi[a] > lo[a])) { err = "invalid periodic box"; return GSPM_E_ARG; }
        M.lo[a] = lo[a];
        M.L[a] = hi[a] - lo[a];
    }
    M.n0 = n0;
    M.ne = ne;

    // ---- 1. periodic identification
    std::vector<std::array<int64_t, 3>> key(static_cast<size_t>(n0));
    std::vector<uint8_t> onmax(static_cast<size_t>(n0), 0);
    for (int64_t i = 0; i < n0; ++i) {
        for (int a = 0; a < 3; ++a) {
            double v = xyz[i * 3 + a], q = 1e-9 * M.L[a];
            if (!std::isfinite(v) || v < lo[a] - q || v > hi[a] + q) { err = "node outside the periodic box"; return GSPM_E_MESH; }
            if (std::fabs(v - hi[a]) <= q) { v = lo[a]; onmax[i] = 1; }
            key[i][a] = std::llround((v - lo[a]) / q);
        }
    }
    std::unordered_map<std::array<int64_t, 3>, int32_t, KeyHash> site;
    site.reserve(static_cast<size_t>(n0));
    std::vector<int32_t> uid(static_cast<size_t>(n0), -1);
    std::vector<int64_t> rep;                                  // unique -> caller's representative node
    for (int64_t i = 0; i < n0; ++i) {
        if (onmax[i]) continue;
        auto ins = site.emplace(key[i], static_cast<int32_t>(rep.size()));
        if (!ins.second) { err = "two nodes share one position"; return GSPM_E_MESH; }
        uid[i] = ins.first->second;
        rep.push_back(i);
    }
    for (int64_t i = 0; i < n0; ++i) {
        if (!onmax[i]) continue;
        auto it = site.find(key[i]);
        if (it == site.end()) { err = "unmatched periodic node on a max face"; return GSPM_E_MESH; }
        uid[i] = it->second;
    }
    const int32_t n = static_cast<int32_t>(rep.size());
    M.n = n;

    // ---- 2. validation, geometry, lumped weights (unique-id indexing)
    std::vector<double> wu(static_cast<size_t>(n), 0.0);
    double vc = 0.0;
    for (int64_t e = 0; e < ne; ++e) {
        int32_t v[4];
        for (int j = 0; j < 4; ++j) {
            int32_t t = tets[e * 4 + j];
            if (t < 0 || t >= n0) { err = "tetrahedron refers to a node that does not exist"; return GSPM_E_MESH; }
            v[j] = uid[t];
        }
        for (int j = 0; j < 4; ++j)
            for (int k = j + 1; k < 4; ++k)
                if (v[j] == v[k]) { err = "tetrahedron with a repeated (periodic) vertex"; return GSPM_E_MESH; }
        double d[3][3], len2 = 0.0;
        for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 3; ++a) {
                double dv = xyz[rep[v[k + 1]] * 3 + a] - xyz[rep[v[0]] * 3 + a];
                dv -= M.L[a] * std::nearbyint(dv / M.L[a]);
                d[k][a] = dv;
                len2 += dv * dv;
            }
        double det = d[0][0] * (d[1][1] * d[2][2] - d[1][2] * d[2][1]) - d[0][1] * (d[1][0] * d[2][2] - d[1][2] * d[2][0]) +
                     d[0][2] * (d[1][0] * d[2][1] - d[1][1] * d[2][0]);
        double vol = std::fabs(det) / 6.0, h = std::sqrt(len2 / 3.0);
        if (!(vol > 1e-9 * h * h * h)) { err = "degenerate tetrahedron"; return GSPM_E_MESH; }
        vc += vol;
        if (tags[e])
            for (int j = 0; j < 4; ++j) wu[v[j]] += 0.25 * vol;
    }
    M.vc = vc;

    // ---- 3. renumbering of the unique nodes: Morton curve (default), the
    // caller's order, or reverse Cuthill-McKee on the mesh graph
    std::vector<int32_t> order(static_cast<size_t>(n));
    std::iota(order.begin(), order.end(), 0);
    if (reorder == GSPM_REORDER_MORTON) {
        std::vector<uint64_t> code(static_cast<size_t>(n));
        for (int32_t g = 0; g < n; ++g) {
            uint64_t c = 0;
            for (int a = 0; a < 3; ++a) {
                double t = (xyz[rep[g] * 3 + a] - lo[a]) / M.L[a];
                t = std::min(std::max(t, 0.0), 1.0 - 1e-12);
                c |= spread3(static_cast<uint64_t>(t * 2097152.0)) << a;
            }
            code[g] = c;
        }
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return code[a] < code[b]; });
    } else if (reorder == GSPM_REORDER_RCM) {
        // node graph (vertices sharing a tetrahedron), breadth-first from a
        // node of least degree, neighbours by increasing degree, reversed
        std::vector<int64_t> deg(static_cast<size_t>(n) + 1, 0);
        for (int64_t e = 0; e < ne; ++e)
            for (int j = 0; j < 4; ++j) deg[static_cast<size_t>(uid[tets[e * 4 + j]]) + 1] += 3;
        for (int32_t g = 0; g < n; ++g) deg[g + 1] += deg[g];
        std::vector<int32_t> adj(static_cast<size_t>(deg[n]));
        std::vector<int64_t> fill(deg.begin(), deg.end() - 1);
        for (int64_t e = 0; e < ne; ++e)
            for (int j = 0; j < 4; ++j)
                for (int k = 0; k < 4; ++k)
                    if (k != j) adj[fill[uid[tets[e * 4 + j]]]++] = uid[tets[e * 4 + k]];
        std::vector<int32_t> nd(static_cast<size_t>(n));
        for (int32_t g = 0; g < n; ++g) {
            auto b = adj.begin() + deg[g], en = adj.begin() + deg[g + 1];
            std::sort(b, en);
            nd[g] = static_cast<int32_t>(std::unique(b, en) - b);
        }
        std::vector<uint8_t> seen(static_cast<size_t>(n), 0);
        std::vector<int32_t> cm;
        cm.reserve(static_cast<size_t>(n));
        std::vector<int32_t> by_deg(order);
        std::stable_sort(by_deg.begin(), by_deg.end(), [&](int32_t a, int32_t b) { return nd[a] < nd[b]; });
        for (int32_t start : by_deg) {          // every connected component
            if (seen[start]) continue;
            seen[start] = 1;
            size_t head = cm.size();
            cm.push_back(start);
            while (head < cm.size()) {
                const int32_t g = cm[head++];
                std::vector<int32_t> next;
                for (int64_t q = deg[g]; q < deg[g] + nd[g]; ++q)
                    if (!seen[adj[q]]) {
                        seen[adj[q]] = 1;
                        next.push_back(adj[q]);
                    }
                std::stable_sort(next.begin(), next.end(), [&](int32_t a, int32_t b) { return nd[a] < nd[b]; });
                cm.insert(cm.end(), next.begin(), next.end());
            }
        }
        std::reverse(cm.begin(), cm.end());
        order = cm;
    } else if (reorder != GSPM_REORDER_NONE) {
        err = "unknown node order";
        return GSPM_E_ARG;
    }
    std::vector<int32_t> newid(static_cast<size_t>(n));
    for (int32_t k = 0; k < n; ++k) newid[order[k]] = k;

    M.user2int.resize(static_cast<size_t>(n0));
    for (int64_t i = 0; i < n0; ++i) M.user2int[i] = newid[uid[i]];
    M.xs.resize(3 * static_cast<size_t>(n));
    M.w.resize(static_cast<size_t>(n));
    for (int32_t g = 0; g < n; ++g) {
        int32_t k = newid[g];
        for (int a = 0; a < 3; ++a) M.xs[static_cast<size_t>(a) * n + k] = xyz[rep[g] * 3 + a];
        M.w[k] = wu[g];
    }
    M.p0 = M.user2int[0];

    // ---- 4. owner blocks and their element lists
    M.nb = nb;
    M.nblk = (n + nb - 1) / nb;
    std::vector<int64_t> cnt(static_cast<size_t>(M.nblk) + 1, 0);
    auto blocks_of = [&](int64_t e, int32_t *blk) {
        int nbk = 0;
        for (int j = 0; j < 4; ++j) {
            int32_t b = M.user2int[tets[e * 4 + j]] / nb;
            bool seen = false;
            for (int k = 0; k < nbk; ++k) seen |= (blk[k] == b);
            if (!seen) blk[nbk++] = b;
        }
        return nbk;
    };
    for (int64_t e = 0; e < ne; ++e) {
        int32_t blk[4];
        int nbk = blocks_of(e, blk);
        for (int k = 0; k < nbk; ++k) cnt[blk[k] + 1]++;
    }
    for (int32_t b = 0; b < M.nblk; ++b) cnt[b + 1] += cnt[b];
    M.ncopies = cnt[M.nblk];
    if (M.ncopies > INT32_MAX) { err = "mesh too large for 32-bit element lists"; return GSPM_E_ARG; }
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    std::vector<int64_t> copy_elem(static_cast<size_t>(M.ncopies));
    for (int64_t e = 0; e < ne; ++e) {
        int32_t blk[4];
        int nbk = blocks_of(e, blk);
        for (int k = 0; k < nbk; ++k) copy_elem[fill[blk[k]]++] = e;
    }
    M.blk_ptr.resize(static_cast<size_t>(M.nblk) + 1);
    M.blk_nmag.resize(static_cast<size_t>(M.nblk));
    M.halo_ptr.assign(static_cast<size_t>(M.nblk) + 1, 0);
    M.halo_lo.resize(static_cast<size_t>(M.nblk));
    M.img.resize(static_cast<size_t>(M.nblk));
    M.lconn.resize(4 * static_cast<size_t>(M.ncopies));
    M.seg_ptr.assign(static_cast<size_t>(M.nblk) + 1, 0);
    M.seg_nmag.assign(static_cast<size_t>(M.nblk), 0);
    M.seg_ent.clear();
    M.seg_off.clear();
    M.seg_nel.clear();
    M.halo_ids.clear();
    M.nloc_max = 0;
    std::vector<int32_t> halo, ord_mag, ord_rest;
    for (int32_t b = 0; b < M.nblk; ++b) {
        const int32_t n0b = b * nb, n1b = std::min(n0b + nb, n);
        M.blk_ptr[b] = static_cast<int32_t>(cnt[b]);
        auto first = copy_elem.begin() + cnt[b], last = copy_elem.begin() + cnt[b + 1];
        auto minv = [&](int64_t e) {
            int32_t m = INT32_MAX;
            for (int j = 0; j < 4; ++j) m = std::min(m, M.user2int[tets[e * 4 + j]]);
            return m;
        };
        std::sort(first, last, [&](int64_t a, int64_t c) {
            bool ma = tags[a] != 0, mc = tags[c] != 0;
            if (ma != mc) return ma;
            int32_t va = minv(a), vb = minv(c);
            return va != vb ? va < vb : a < c;
        });
        int32_t nmag = 0;
        for (auto it = first; it != last; ++it) nmag += tags[*it] != 0;
        M.blk_nmag[b] = nmag;
        // halo: vertices of the block's elements outside its owned range
        halo.clear();
        for (auto it = first; it != last; ++it)
            for (int j = 0; j < 4; ++j) {
                const int32_t v = M.user2int[tets[*it * 4 + j]];
                if (v < n0b || v >= n1b) halo.push_back(v);
            }
        std::sort(halo.begin(), halo.end());
        halo.erase(std::unique(halo.begin(), halo.end()), halo.end());
        const int32_t nloc = nb + static_cast<int32_t>(halo.size());
        if (nloc > kMaxLocal) { err = "element block too large for 13-bit local indices"; return GSPM_E_ARG; }
        M.nloc_max = std::max(M.nloc_max, nloc);
        M.halo_lo[b] = static_cast<int32_t>(std::lower_bound(halo.begin(), halo.end(), n0b) - halo.begin());
        M.halo_ptr[b + 1] = M.halo_ptr[b] + static_cast<int32_t>(halo.size());
        for (int64_t c = cnt[b]; c < cnt[b + 1]; ++c)
            for (int j = 0; j < 4; ++j) {
                const int32_t v = M.user2int[tets[copy_elem[c] * 4 + j]];
                int32_t l = (v >= n0b && v < n1b) ? v - n0b
                                                  : nb + static_cast<int32_t>(std::lower_bound(halo.begin(), halo.end(), v) - halo.begin());
                M.lconn[4 * c + j] = static_cast<uint16_t>(l);
            }
        // Staged coordinates are shifted to the nearest image of the block's
        // first node; if every staged node lies within a quarter box of it,
        // element edges are plain differences of staged coordinates.
        bool far = false;
        auto check = [&](int32_t v) {
            for (int a = 0; a < 3; ++a) {
                double d = M.xs[static_cast<size_t>(a) * n + v] - M.xs[static_cast<size_t>(a) * n + n0b];
                d -= M.L[a] * std::nearbyint(d / M.L[a]);
                far |= std::fabs(d) >= 0.25 * M.L[a];
            }
        };
        for (int32_t v = n0b; v < n1b; ++v) check(v);
        for (int32_t v : halo) check(v);
        M.img[b] = far ? 1 : 0;
        M.halo_ids.insert(M.halo_ids.end(), halo.begin(), halo.end());
        // strips: magnetic elements, then the rest; the smallest update budget
        // per segment that fits the block into kThreads segments (one per
        // thread of the operator kernels, all of about the same length)
        const uint16_t *lc = M.lconn.data() + 4 * cnt[b];
        const uint16_t *lc_rest = lc + 4 * static_cast<size_t>(nmag);
        const int32_t nall = static_cast<int32_t>(cnt[b + 1] - cnt[b]);
        strip_order(lc, nmag, ord_mag);
        strip_order(lc_rest, nall - nmag, ord_rest);
        auto nsegs = [&](int budget) {
            return pack_strips(lc, ord_mag, budget, false, M.seg_ent, M.seg_off, M.seg_nel) +
                   pack_strips(lc_rest, ord_rest, budget, false, M.seg_ent, M.seg_off, M.seg_nel);
        };
        int hi_b = 16;
        while (nsegs(hi_b) > kThreads) hi_b *= 2;   // one element always fits: the loop ends
        int lo_b = std::max(4, hi_b / 2 + 1);
        if (hi_b == 16) lo_b = 4;
        while (lo_b < hi_b) {
            const int mid = (lo_b + hi_b) / 2;
            if (nsegs(mid) <= kThreads) hi_b = mid;
            else lo_b = mid + 1;
        }
        lo_b = hi_b;
        M.seg_ptr[b] = static_cast<int32_t>(M.seg_nel.size());
        pack_strips(lc, ord_mag, lo_b, true, M.seg_ent, M.seg_off, M.seg_nel);
        M.seg_nmag[b] = static_cast<int32_t>(M.seg_nel.size()) - M.seg_ptr[b];
        pack_strips(lc_rest, ord_rest, lo_b, true, M.seg_ent, M.seg_off, M.seg_nel);
    }
    M.blk_ptr[M.nblk] = static_cast<int32_t>(M.ncopies);
    M.seg_ptr[M.nblk] = static_cast<int32_t>(M.seg_nel.size());
    M.seg_ent.resize(M.seg_ent.size() + 16, 0);   // lookahead of the operator kernels stays in bounds
    M.nhalo = static_cast<int64_t>(M.halo_ids.size());
    return GSPM_OK;
}

}  // namespace gspm
