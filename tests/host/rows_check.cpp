// Host check of the GS operator's rows built at mesh upload (gs_rows.cpp).
// Decodes the sliced layout back to global columns and checks that
//   - every column index addresses a staged node of the row's block, padding
//     entries point at the row itself with zero coefficients, and no entry
//     lies outside its slice;
//   - (eps K + M) x from the decoded rows equals the same product summed
//     element by element over the magnetic tets (geometry recomputed here from
//     the caller's coordinates), for random x;
//   - K and M are symmetric, K's rows sum to zero, and M's entries sum to the
//     magnetic volume.
//   - each row block's halo list is sorted, lies outside the block's owned
//     range and holds only nodes that some row of the block uses.
// Usage: rows_check <mesh.bin> <block_nodes> [reorder] [row_block_nodes]; prints statistics, exit 0 if valid.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <string>
#include <vector>

#include "common.h"
using namespace gspm;

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    FILE *fp = fopen(argv[1], "rb");
    if (!fp) return 2;
    int64_t n0, ne;
    double lo[3], hi[3];
    size_t got = 0;
    got += fread(&n0, 8, 1, fp);
    got += fread(&ne, 8, 1, fp);
    got += fread(lo, 8, 3, fp);
    got += fread(hi, 8, 3, fp);
    std::vector<double> xyz(3 * n0);
    std::vector<int32_t> tets(4 * ne);
    std::vector<uint8_t> tags(ne);
    got += fread(xyz.data(), 8, 3 * n0, fp);
    got += fread(tets.data(), 4, 4 * ne, fp);
    got += fread(tags.data(), 1, ne, fp);
    fclose(fp);
    if (got != static_cast<size_t>(8 + 3 * n0 + 4 * ne + ne)) {
        printf("short mesh file\n");
        return 2;
    }
    const int nb = argc > 2 ? atoi(argv[2]) : 256;
    const int reorder = argc > 3 ? atoi(argv[3]) : GSPM_REORDER_MORTON;
    const int nb_rows = argc > 4 ? atoi(argv[4]) : 0;
    HostMesh M;
    std::string err;
    if (prepare_mesh(n0, xyz.data(), ne, tets.data(), tags.data(), lo, hi, nb, M, err, reorder)) {
        printf("prepare failed %s\n", err.c_str());
        return 1;
    }
    GsRowsHost R;
    if (assemble_gs_rows(M, ne, tets.data(), tags.data(), nb_rows, R, err)) {
        printf("assembly failed %s\n", err.c_str());
        return 1;
    }
    const int n = M.n;
    long bad = 0;
    const int rb = R.nb;
    if (rb != (nb_rows > 0 ? nb_rows : M.nb) || R.nblk != (n + rb - 1) / rb ||
        static_cast<int>(R.halo_ptr.size()) != R.nblk + 1 ||
        static_cast<size_t>(R.halo_ptr[R.nblk]) != R.halo_ids.size()) {
        printf("row blocks inconsistent\n");
        return 1;
    }
    std::vector<char> used(R.halo_ids.size(), 0);
    const int nsl = (n + 63) / 64;
    if (static_cast<int>(R.off.size()) != nsl + 1 || R.off[0] != 0 ||
        static_cast<size_t>(R.off[nsl]) != R.col.size()) {
        printf("slice offsets inconsistent\n");
        return 1;
    }
    // decode
    std::vector<std::map<int, std::pair<double, double>>> rows(n);
    long entries = 0, padding = 0;
    for (int i = 0; i < n; ++i) {
        const int b = i / rb, nloc = rb + (R.halo_ptr[b + 1] - R.halo_ptr[b]);
        const int s = i / 64, lane = i % 64, w = (R.off[s + 1] - R.off[s]) / 64;
        if ((R.off[s + 1] - R.off[s]) % 64) bad++;
        for (int k = 0; k < w; ++k) {
            const size_t e = static_cast<size_t>(R.off[s]) + 64 * static_cast<size_t>(k) + lane;
            const int loc = R.col[e];
            if (loc >= nloc || (loc >= n - b * rb && loc < rb)) {
                bad++;
                printf("row %d: column %d outside the staged set\n", i, loc);
                continue;
            }
            if (loc >= rb) used[R.halo_ptr[b] + loc - rb] = 1;
            const int j = loc < rb ? b * rb + loc : R.halo_ids[R.halo_ptr[b] + loc - rb];
            if (j == i) {
                if (R.kv[e] != 0.0 || R.mv[e] != 0.0) {
                    bad++;
                    printf("row %d: padding with a coefficient\n", i);
                }
                padding++;
                continue;
            }
            if (rows[i].count(j)) {
                bad++;
                printf("row %d: column %d twice\n", i, j);
            }
            rows[i][j] = {R.kv[e], R.mv[e]};
            entries++;
        }
    }
    // symmetry, zero row sums of K, total mass
    double kscale = 0.0, vmag = 0.0, msum = 0.0, worst_sym = 0.0, worst_rowsum = 0.0;
    for (int i = 0; i < n; ++i) kscale = std::max(kscale, std::fabs(R.kd[i]));
    for (int i = 0; i < n; ++i) {
        double rs = R.kd[i];
        msum += R.md[i];
        for (auto &kv : rows[i]) {
            rs += kv.second.first;
            msum += kv.second.second;
            auto it = rows[kv.first].find(i);
            if (it == rows[kv.first].end()) {
                bad++;
                printf("entry (%d, %d) has no transpose\n", i, kv.first);
                continue;
            }
            worst_sym = std::max(worst_sym, std::fabs(it->second.first - kv.second.first) / kscale);
            worst_sym = std::max(worst_sym, std::fabs(it->second.second - kv.second.second) / kscale);
        }
        worst_rowsum = std::max(worst_rowsum, std::fabs(rs) / kscale);
    }
    // element-by-element product
    std::mt19937_64 gen(7);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    const double eps = 0.37 * std::cbrt(M.vc / ne) * std::cbrt(M.vc / ne);
    std::vector<double> x(n), y1(n, 0.0), y2(n, 0.0);
    for (auto &v : x) v = U(gen);
    const double L[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
    for (int64_t e = 0; e < ne; ++e) {
        if (!tags[e]) continue;
        const int32_t *t = tets.data() + 4 * e;
        double E[3][3];
        for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 3; ++a) {
                double d = xyz[3 * t[k + 1] + a] - xyz[3 * t[0] + a];
                d -= L[a] * std::nearbyint(d / L[a]);
                E[k][a] = d;
            }
        // gradients by solving E g = unit vectors (Cramer's rule)
        const double det = E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) -
                           E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
                           E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
        const double V = std::fabs(det) / 6.0;
        double inv[3][3];   // inverse of E; column k is grad lambda_{k+1}
        inv[0][0] = (E[1][1] * E[2][2] - E[1][2] * E[2][1]) / det;
        inv[0][1] = (E[0][2] * E[2][1] - E[0][1] * E[2][2]) / det;
        inv[0][2] = (E[0][1] * E[1][2] - E[0][2] * E[1][1]) / det;
        inv[1][0] = (E[1][2] * E[2][0] - E[1][0] * E[2][2]) / det;
        inv[1][1] = (E[0][0] * E[2][2] - E[0][2] * E[2][0]) / det;
        inv[1][2] = (E[0][2] * E[1][0] - E[0][0] * E[1][2]) / det;
        inv[2][0] = (E[1][0] * E[2][1] - E[1][1] * E[2][0]) / det;
        inv[2][1] = (E[0][1] * E[2][0] - E[0][0] * E[2][1]) / det;
        inv[2][2] = (E[0][0] * E[1][1] - E[0][1] * E[1][0]) / det;
        double g[4][3];
        for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 3; ++a) g[k + 1][a] = inv[a][k];
        for (int a = 0; a < 3; ++a) g[0][a] = -(g[1][a] + g[2][a] + g[3][a]);
        int v[4];
        for (int j = 0; j < 4; ++j) v[j] = M.user2int[t[j]];
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                const double k = V * (g[i][0] * g[j][0] + g[i][1] * g[j][1] + g[i][2] * g[j][2]);
                const double m = V * (i == j ? 2.0 : 1.0) / 20.0;
                y1[v[i]] += (eps * k + m) * x[v[j]];
            }
        vmag += V;
    }
    double ynorm = 0.0, dnorm = 0.0;
    for (int i = 0; i < n; ++i) {
        double acc = (eps * R.kd[i] + R.md[i]) * x[i];
        for (auto &kv : rows[i]) acc += (eps * kv.second.first + kv.second.second) * x[kv.first];
        y2[i] = acc;
        ynorm += y1[i] * y1[i];
        dnorm += (y1[i] - y2[i]) * (y1[i] - y2[i]);
    }
    // halo lists: sorted, outside the owned range, every entry used
    long halo_bad = 0;
    for (int b = 0; b < R.nblk; ++b)
        for (int t = R.halo_ptr[b]; t < R.halo_ptr[b + 1]; ++t) {
            const int j = R.halo_ids[t];
            if ((t > R.halo_ptr[b] && R.halo_ids[t - 1] >= j) || (j >= b * rb && j < (b + 1) * rb) || !used[t])
                halo_bad++;
        }
    if (halo_bad) {
        bad++;
        printf("%ld halo entries unsorted, owned or unused\n", halo_bad);
    }
    const double rel = std::sqrt(dnorm / ynorm), mrel = std::fabs(msum - vmag) / vmag;
    printf("rows %d entries %ld padding %ld (%.1f%%) per row %.2f | row blocks of %d: %.2f halo nodes per row | "
           "product rel err %.2e | symmetry %.1e row sums %.1e mass %.1e\n",
           n, entries, padding, 100.0 * padding / std::max(1L, entries + padding), double(entries) / n, rb,
           double(R.halo_ids.size()) / n, rel, worst_sym, worst_rowsum, mrel);
    if (rel > 1e-13 || worst_sym > 1e-13 || worst_rowsum > 1e-12 || mrel > 1e-13) bad++;
    return bad ? 1 : 0;
}
