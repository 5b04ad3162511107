// Host check of the tet-strip encoding built at mesh upload (mesh_prep.cpp):
// decoding every block's segments with a four-slot window must reproduce the
// block's element list exactly (as a multiset of vertex sets, magnetic and
// non-magnetic groups apart), every local id must index a staged node, and
// the mask must mark only entries of the segment.
// Usage: strip_check <mesh.bin> <block_nodes>; prints statistics, exit 0 if valid.
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
    HostMesh M; std::string err;
    int rc = prepare_mesh(n0, xyz.data(), ne, tets.data(), tags.data(), lo, hi, nb, M, err);
    if (rc) { printf("prepare failed %s\n", err.c_str()); return 1; }
    long bad = 0, loads = 0, elems = 0, flush = 0;
    for (int b = 0; b < M.nblk; ++b) {
        const int nloc = M.nb + (M.halo_ptr[b + 1] - M.halo_ptr[b]);
        std::map<std::array<int,4>, int> want[2], got[2];
        for (int e = M.blk_ptr[b]; e < M.blk_ptr[b + 1]; ++e) {
            std::array<int,4> v{M.lconn[4*e], M.lconn[4*e+1], M.lconn[4*e+2], M.lconn[4*e+3]};
            std::sort(v.begin(), v.end());
            want[(e - M.blk_ptr[b]) < M.blk_nmag[b] ? 0 : 1][v]++;
        }
        for (int s = M.seg_ptr[b]; s < M.seg_ptr[b + 1]; ++s) {
            int grp = (s - M.seg_ptr[b]) < M.seg_nmag[b] ? 0 : 1;
            int win[4] = {-1, -1, -1, -1};
            unsigned msk = M.seg_mask[s];
            bool ended = false;
            for (int k = 0; k < kSegEntries; ++k) {
                unsigned e = M.seg_ent[s * kSegEntries + k];
                if (e == kSegEnd) { ended = true; continue; }
                if (ended) { bad++; printf("entry after end\n"); }
                int id = e & 0x3FFF, sl = e >> 14;
                if (id >= nloc) { bad++; printf("id %d >= nloc %d\n", id, nloc); }
                if (win[sl] >= 0 && win[sl] < M.nb) flush++;
                win[sl] = id; loads++;
                if (msk >> k & 1) {
                    std::array<int,4> v{win[0], win[1], win[2], win[3]};
                    std::sort(v.begin(), v.end());
                    if (v[0] < 0 || v[0] == v[1] || v[1] == v[2] || v[2] == v[3]) { bad++; printf("bad window\n"); }
                    got[grp][v]++; elems++;
                }
            }
            if ((msk >> kSegEntries) != 0) bad++;
            for (int j = 0; j < 4; ++j) if (win[j] >= 0 && win[j] < M.nb) flush++;
        }
        for (int g = 0; g < 2; ++g) if (want[g] != got[g]) { bad++; printf("block %d group %d mismatch %zu vs %zu\n", b, g, want[g].size(), got[g].size()); }
    }
    printf("blocks %d copies %lld segments %zu elems %ld loads/elem %.3f owned flushes/elem %.3f segs/block %.1f bad %ld\n",
           M.nblk, (long long)M.ncopies, M.seg_mask.size(), elems, double(loads)/elems, double(flush)/elems,
           double(M.seg_mask.size())/M.nblk, bad);
    return bad ? 2 : 0;
}
