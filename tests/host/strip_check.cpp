// Host check of the tet-strip encoding built at mesh upload (mesh_prep.cpp):
// decoding every block's segments with a four-slot window must reproduce the
// block's element list exactly (as a multiset of vertex sets, magnetic and
// non-magnetic groups apart), every local id must index a staged node, every
// segment must stay inside its entries, and no block may have more segments
// than a workgroup has threads.
// Usage: strip_check <mesh.bin> <block_nodes> [reorder]; prints statistics, exit 0 if valid.
#include <algorithm>
#include <cstdio>
#include <map>
#include <vector>
#include <array>
#include <cstdlib>
#include <string>

#include "common.h"
using namespace gspm;
int main(int argc, char **argv) {
    FILE *fp = fopen(argv[1], "rb");
    int64_t n0, ne; double lo[3], hi[3];
    fread(&n0, 8, 1, fp); fread(&ne, 8, 1, fp); fread(lo, 8, 3, fp); fread(hi, 8, 3, fp);
    std::vector<double> xyz(3 * n0); std::vector<int32_t> tets(4 * ne); std::vector<uint8_t> tags(ne);
    fread(xyz.data(), 8, 3 * n0, fp); fread(tets.data(), 4, 4 * ne, fp); fread(tags.data(), 1, ne, fp); fclose(fp);
    int nb = argc > 2 ? atoi(argv[2]) : 256;
    int reorder = argc > 3 ? atoi(argv[3]) : GSPM_REORDER_MORTON;
    HostMesh M; std::string err;
    int rc = prepare_mesh(n0, xyz.data(), ne, tets.data(), tags.data(), lo, hi, nb, M, err, reorder);
    if (rc) { printf("prepare failed %s\n", err.c_str()); return 1; }
    long bad = 0, loads = 0, elems = 0, flush = 0, segs_total = 0;
    for (int b = 0; b < M.nblk; ++b) {
        const int nloc = M.nb + (M.halo_ptr[b + 1] - M.halo_ptr[b]);
        std::map<std::array<int,4>, int> want[2], got[2];
        for (int e = M.blk_ptr[b]; e < M.blk_ptr[b + 1]; ++e) {
            std::array<int,4> v{M.lconn[4*e], M.lconn[4*e+1], M.lconn[4*e+2], M.lconn[4*e+3]};
            std::sort(v.begin(), v.end());
            want[(e - M.blk_ptr[b]) < M.blk_nmag[b] ? 0 : 1][v]++;
        }
        int maxnel = 0, minnel = 1 << 30;
        for (int s = M.seg_ptr[b]; s < M.seg_ptr[b + 1]; ++s) {
            int grp = (s - M.seg_ptr[b]) < M.seg_nmag[b] ? 0 : 1;
            int win[4] = {-1, -1, -1, -1};
            size_t k = 8 * static_cast<size_t>(M.seg_off[s]);
            const size_t kend = s + 1 < static_cast<int>(M.seg_off.size()) ? 8 * static_cast<size_t>(M.seg_off[s + 1])
                                                                            : M.seg_ent.size() - 16;
            // the kernels read two uint4 ahead of the entries they consume
            if (8 * static_cast<size_t>(M.seg_off[s]) + 16 > M.seg_ent.size()) { bad++; printf("lookahead out of range\n"); }
            if (k % 8) { bad++; printf("unaligned segment\n"); }
            const int nent = M.seg_nel[s];
            maxnel = std::max(maxnel, nent); minnel = std::min(minnel, nent);
            if (k + nent > kend) { bad++; printf("segment overrun\n"); continue; }
            // the operator kernels load the first element of a segment straight
            // into slots 0..3: its four entries take those slots in order, and
            // only the fourth completes an element
            if (nent < 4) { bad++; printf("segment shorter than one element\n"); }
            for (int i = 0; i < 4 && i < nent; ++i) {
                unsigned e = M.seg_ent[k + i];
                if ((e >> 14) != static_cast<unsigned>(i) || ((e & kEntElem) != 0) != (i == 3)) {
                    bad++; printf("segment does not open with slots 0..3\n"); break;
                }
            }
            for (int i = 0; i < nent; ++i) {
                unsigned e = M.seg_ent[k++];
                int id = e & kEntIdMask, sl = e >> 14;
                if (id >= nloc) { bad++; printf("id %d >= nloc %d\n", id, nloc); }
                if (i < 4) {
                    win[i] = id;                               // the opening element fills slots 0..3
                } else {
                    if (win[sl] >= 0 && win[sl] < M.nb) flush++;
                    win[sl] = win[3];                          // slot 3 moves into the freed slot
                    win[3] = id;                               // the new vertex takes slot 3
                }
                loads++;
                if (e & kEntElem) {
                    std::array<int,4> v{win[0], win[1], win[2], win[3]};
                    std::sort(v.begin(), v.end());
                    if (v[0] < 0 || v[0] == v[1] || v[1] == v[2] || v[2] == v[3]) { bad++; printf("bad window\n"); }
                    got[grp][v]++; elems++;
                } else if (i == nent - 1) { bad++; printf("segment ends inside an element\n"); }
            }
            for (int j = 0; j < 4; ++j) if (win[j] >= 0 && win[j] < M.nb) flush++;
        }
        if (M.seg_ptr[b + 1] - M.seg_ptr[b] > kThreads) { bad++; printf("block %d has %d segments\n", b, M.seg_ptr[b + 1] - M.seg_ptr[b]); }
        segs_total += M.seg_ptr[b + 1] - M.seg_ptr[b];
        (void)maxnel; (void)minnel;
        for (int g = 0; g < 2; ++g) if (want[g] != got[g]) { bad++; printf("block %d group %d mismatch %zu vs %zu\n", b, g, want[g].size(), got[g].size()); }
    }
    printf("blocks %d copies %lld segments %ld elems %ld loads/elem %.3f owned flushes/elem %.3f segs/block %.1f bad %ld\n",
           M.nblk, (long long)M.ncopies, segs_total, elems, double(loads)/elems, double(flush)/elems,
           double(segs_total)/M.nblk, bad);
    return bad ? 2 : 0;
}
