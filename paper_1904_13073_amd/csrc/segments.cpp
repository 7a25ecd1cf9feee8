// Host-side layout of the segment Gram storage (plain C++, no HIP).
#include "segments.h"

#include <algorithm>

namespace swgn {

namespace {

inline int first_pair(int pa) { return 5 * pa - pa * (pa - 1) / 2; }

void decode_key(uint64_t k, int* t) {
    t[0] = (int)(k >> 48);
    t[1] = (int)((k >> 32) & 0xffff);
    t[2] = (int)((k >> 16) & 0xffff);
    t[3] = (int)(k & 0xffff);
}

}  // namespace

bool segment_layout_sets(int nsets, const uint64_t* set_key, const int* set_start, int nn, int nb,
                         const int* row_ptr, const int* col_idx, int max_surfels, SegmentLayout& L,
                         std::string& why) {
    L = SegmentLayout{};
    if (nsets < 0 || nn <= 0 || nb < nn || max_surfels <= 0 || (nsets > 0 && set_start[0] != 0)) {
        why = "segment layout: bad sizes";
        return false;
    }
    // greedy segments whose node union stays within 5 nodes and max_surfels
    // surfels; within a run of one node set only the length can cut, so the
    // walk is per run: a run that does not fit starts a segment, a long one is
    // cut every max_surfels surfels
    std::vector<uint64_t> seg_sets;      // node sets of the open segment
    std::vector<int> seg_set_ptr{0};     // per closed segment: its range in all_sets
    std::vector<uint64_t> all_sets;
    int cur[5] = {-1, -1, -1, -1, -1}, cn = 0, start = 0;
    auto close = [&]() {
        L.seg_start.push_back(start);
        for (int q = 0; q < 5; ++q) L.seg_nodes.push_back(q < cn ? cur[q] : -1);
        all_sets.insert(all_sets.end(), seg_sets.begin(), seg_sets.end());
        seg_set_ptr.push_back((int)all_sets.size());
        seg_sets.clear();
    };
    for (int r = 0; r < nsets; ++r) {
        int t[4];
        decode_key(set_key[r], t);
        for (int k = 0; k < 4; ++k)
            if (t[k] >= nn || (k > 0 && t[k] <= t[k - 1])) {
                why = "segment layout: a node set is not 4 distinct ascending nodes";
                return false;
            }
        const int a = set_start[r], b = set_start[r + 1];
        if (b <= a || (r > 0 && set_key[r] <= set_key[r - 1])) {
            why = "segment layout: node-set runs are empty or not ascending";
            return false;
        }
        // union of the segment's nodes and t, ascending; at most 5 + 4 entries
        int u[9], un = 0, x = 0, y = 0;
        while (x < cn || y < 4) {
            int v;
            if (y >= 4 || (x < cn && cur[x] < t[y])) v = cur[x++];
            else if (x >= cn || t[y] < cur[x]) v = t[y++];
            else { v = cur[x++]; ++y; }
            u[un++] = v;
        }
        if (r == 0 || un > 5 || a - start >= max_surfels) {
            if (r > 0) close();
            start = a;
            cn = 4;
            for (int q = 0; q < 4; ++q) cur[q] = t[q];
        } else {
            cn = un;
            for (int q = 0; q < un; ++q) cur[q] = u[q];
        }
        seg_sets.push_back(set_key[r]);
        while (b - start > max_surfels) {
            close();
            start += max_surfels;
            cn = 4;
            for (int q = 0; q < 4; ++q) cur[q] = t[q];
            seg_sets.push_back(set_key[r]);
        }
    }
    if (nsets > 0) close();
    const int nseg = (int)L.seg_start.size();
    const int ns = nsets > 0 ? set_start[nsets] : 0;
    L.seg_start.push_back(ns);

    // pair mask (from the node sets a segment holds) and offset of each segment
    L.mask.assign(nseg, 0);
    L.off.assign(nseg + 1, 0);
    uint64_t total = 0;
    for (int g = 0; g < nseg; ++g) {
        const int* nd = &L.seg_nodes[5 * g];
        uint32_t m = 0;
        for (int q = seg_set_ptr[g]; q < seg_set_ptr[g + 1]; ++q) {
            int t[4], p[4];
            decode_key(all_sets[q], t);
            for (int k = 0; k < 4; ++k) {
                p[k] = 0;
                while (p[k] < 5 && nd[p[k]] != t[k]) ++p[k];
            }
            for (int x = 0; x < 4; ++x)
                for (int y = 0; y < 4; ++y)
                    if (p[x] <= p[y]) m |= 1u << (first_pair(p[x]) + p[y] - p[x]);
        }
        L.mask[g] = (uint16_t)m;
        L.off[g] = (uint32_t)total;
        total += 36u * (uint64_t)__builtin_popcount(m) + 32u;
        if (total >= (1ull << 32)) {
            why = "segment Gram storage exceeds 2^32 floats";
            return false;
        }
    }
    L.off[nseg] = (uint32_t)total;
    L.total = total;

    // entries of every block in segment order (a counting sort by block)
    struct Ent { int blk; uint32_t sub, grad; };
    std::vector<Ent> ents;
    ents.reserve((size_t)nseg * 10);
    for (int g = 0; g < nseg; ++g) {
        const int* nd = &L.seg_nodes[5 * g];
        const uint32_t m = L.mask[g];
        const uint32_t np = (uint32_t)__builtin_popcount(m);
        uint32_t rank = 0;
        for (int pa = 0; pa < 5; ++pa)
            for (int pb = pa; pb < 5; ++pb) {
                if (!((m >> (first_pair(pa) + pb - pa)) & 1u)) continue;
                const int ra = nd[pa], cb = nd[pb];
                const int* lo = col_idx + row_ptr[ra];
                const int* hi = col_idx + row_ptr[ra + 1];
                const int* at = std::lower_bound(lo, hi, cb);
                if (at == hi || *at != cb) {
                    why = "segment layout: the block pattern misses a node pair";
                    return false;
                }
                const uint32_t grad = pa == pb ? L.off[g] + 36u * np + 6u * (uint32_t)pa : 0xffffffffu;
                ents.push_back(Ent{(int)(at - col_idx), L.off[g] + 36u * rank, grad});
                ++rank;
            }
    }
    L.ent_ptr.assign(nb + 1, 0);
    for (const Ent& e : ents) L.ent_ptr[e.blk + 1] += 1;
    for (int b = 0; b < nb; ++b) L.ent_ptr[b + 1] += L.ent_ptr[b];
    L.ent_sub.resize(ents.size());
    L.ent_grad.resize(ents.size());
    std::vector<int> fill(L.ent_ptr.begin(), L.ent_ptr.end() - 1);
    for (const Ent& e : ents) {
        const int at = fill[e.blk]++;
        L.ent_sub[at] = e.sub;
        L.ent_grad[at] = e.grad;
    }

    // packs of whole segments
    L.pack_start.assign(1, 0);
    L.pack_seg.assign(1, 0);
    for (int g = 0; g < nseg; ++g)
        if (L.seg_start[g + 1] - L.pack_start.back() > max_surfels) {
            L.pack_start.push_back(L.seg_start[g]);
            L.pack_seg.push_back(g);
        }
    L.pack_start.push_back(ns);
    L.pack_seg.push_back(nseg);
    return true;
}

bool segment_layout(int ns, int nn, int nb, const uint64_t* key, const int32_t* idx4, const int* row_ptr,
                    const int* col_idx, int max_surfels, SegmentLayout& L, std::string& why) {
    if (ns < 0) {
        why = "segment layout: bad sizes";
        return false;
    }
    // runs of equal keys
    std::vector<uint64_t> set_key;
    std::vector<int> set_start;
    for (int i = 0; i < ns; ++i) {
        if (i > 0 && key[i] < key[i - 1]) {
            why = "segment layout: surfels are not sorted by node set";
            return false;
        }
        if (i == 0 || key[i] != key[i - 1]) {
            set_key.push_back(key[i]);
            set_start.push_back(i);
        }
    }
    set_start.push_back(ns);
    if (!segment_layout_sets((int)set_key.size(), set_key.data(), set_start.data(), nn, nb, row_ptr, col_idx,
                             max_surfels, L, why))
        return false;
    // positions of each surfel's nodes among its segment's nodes
    L.pos4.assign(ns, 0);
    const int nseg = (int)L.seg_start.size() - 1;
    for (int g = 0; g < nseg; ++g) {
        const int* nd = &L.seg_nodes[5 * g];
        for (int i = L.seg_start[g]; i < L.seg_start[g + 1]; ++i) {
            int p[4];
            for (int k = 0; k < 4; ++k) {
                const int id = idx4[4 * (int64_t)i + k];
                p[k] = 0;
                while (p[k] < 5 && nd[p[k]] != id) ++p[k];
                if (p[k] == 5) {
                    why = "segment layout: a surfel's slot nodes differ from its node set";
                    return false;
                }
            }
            L.pos4[i] = (uint16_t)(p[0] | (p[1] << 3) | (p[2] << 6) | (p[3] << 9));
        }
    }
    return true;
}

}  // namespace swgn
