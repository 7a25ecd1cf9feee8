// Host check of the segment layout: builds node sets, calls segment_layout and
// verifies every property the correspondence kernel and the block fold rely
// on. Built with AddressSanitizer and UBSan by tests/test_segments_host.py.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <map>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "segments.h"

using swgn::SegmentLayout;

static int failures = 0;
#define CHECK(c, ...)                                          \
    do {                                                       \
        if (!(c)) {                                            \
            if (failures < 20) {                               \
                fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
                fprintf(stderr, __VA_ARGS__);                  \
                fputc('\n', stderr);                           \
            }                                                  \
            ++failures;                                        \
        }                                                      \
    } while (0)

struct Problem {
    int nn = 0;
    std::vector<uint64_t> key;
    std::vector<int32_t> idx4;
    std::vector<int> row_ptr, col_idx;
};

static uint64_t pack4(const int* t) {
    return ((uint64_t)t[0] << 48) | ((uint64_t)t[1] << 32) | ((uint64_t)t[2] << 16) | (uint64_t)t[3];
}

// Sort surfels by node set and build the upper pattern: every node's diagonal
// and every pair of every node set.
static Problem make_problem(int nn, std::vector<std::vector<int>> sets, std::mt19937& rng) {
    Problem P;
    P.nn = nn;
    std::sort(sets.begin(), sets.end(), [](const std::vector<int>& a, const std::vector<int>& b) {
        std::vector<int> x = a, y = b;
        std::sort(x.begin(), x.end());
        std::sort(y.begin(), y.end());
        return x < y;
    });
    std::vector<std::set<int>> rows(nn);
    for (int i = 0; i < nn; ++i) rows[i].insert(i);
    for (auto& s : sets) {
        std::vector<int> t = s;
        std::sort(t.begin(), t.end());
        P.key.push_back(pack4(t.data()));
        std::vector<int> slot = s;
        std::shuffle(slot.begin(), slot.end(), rng);
        for (int k = 0; k < 4; ++k) P.idx4.push_back(slot[k]);
        for (int a = 0; a < 4; ++a)
            for (int b = a; b < 4; ++b) rows[t[a]].insert(t[b]);
    }
    P.row_ptr.push_back(0);
    for (int i = 0; i < nn; ++i) {
        for (int c : rows[i]) P.col_idx.push_back(c);
        P.row_ptr.push_back((int)P.col_idx.size());
    }
    return P;
}

static int first_pair(int pa) { return 5 * pa - pa * (pa - 1) / 2; }

static void unpack_key(uint64_t k, int* t) {
    t[0] = (int)(k >> 48); t[1] = (int)((k >> 32) & 0xffff); t[2] = (int)((k >> 16) & 0xffff); t[3] = (int)(k & 0xffff);
}

static void verify(const Problem& P, int max_surfels, const SegmentLayout& L, const char* name) {
    const int ns = (int)P.key.size(), nb = (int)P.col_idx.size();
    const int nseg = (int)L.mask.size();
    CHECK((int)L.seg_start.size() == nseg + 1, "%s: seg_start size", name);
    CHECK(L.seg_start.front() == 0 && L.seg_start.back() == ns, "%s: segments cover the surfels", name);
    CHECK((int)L.pos4.size() == ns && (int)L.off.size() == nseg + 1, "%s: sizes", name);
    // block id of (row, col) in the upper pattern
    auto block = [&](int r, int c) {
        for (int b = P.row_ptr[r]; b < P.row_ptr[r + 1]; ++b)
            if (P.col_idx[b] == c) return b;
        return -1;
    };
    std::map<int, std::vector<std::pair<uint32_t, uint32_t>>> expect;   // block -> (sub, grad) in segment order
    uint64_t total = 0;
    for (int g = 0; g < nseg; ++g) {
        const int s0 = L.seg_start[g], s1 = L.seg_start[g + 1];
        CHECK(s1 > s0 && s1 - s0 <= max_surfels, "%s: segment %d length %d", name, g, s1 - s0);
        std::set<int> uni;
        for (int i = s0; i < s1; ++i) {
            int t[4];
            unpack_key(P.key[i], t);
            uni.insert(t, t + 4);
        }
        CHECK(uni.size() <= 5, "%s: segment %d has %zu nodes", name, g, uni.size());
        const std::vector<int> nd(uni.begin(), uni.end());
        // greedy: the next surfel would overflow 5 nodes or the length cap
        if (s1 < ns) {
            int t[4];
            unpack_key(P.key[s1], t);
            std::set<int> more = uni;
            more.insert(t, t + 4);
            CHECK(more.size() > 5 || s1 - s0 >= max_surfels, "%s: segment %d ends early", name, g);
        }
        uint32_t m = 0;
        for (int i = s0; i < s1; ++i) {
            int p[4];
            for (int k = 0; k < 4; ++k) {
                p[k] = (L.pos4[i] >> (3 * k)) & 7;
                CHECK(p[k] < (int)nd.size() && nd[p[k]] == P.idx4[4 * i + k], "%s: surfel %d slot %d", name, i, k);
            }
            CHECK((L.pos4[i] >> 12) == 0, "%s: pos4 high bits", name);
            for (int x = 0; x < 4; ++x)
                for (int y = 0; y < 4; ++y)
                    if (p[x] <= p[y]) m |= 1u << (first_pair(p[x]) + p[y] - p[x]);
        }
        CHECK(L.mask[g] == m, "%s: segment %d mask %x != %x", name, g, L.mask[g], m);
        CHECK(L.off[g] == total, "%s: segment %d offset", name, g);
        const int np = __builtin_popcount(m);
        total += 36u * np + 32u;
        int rank = 0;
        for (int pa = 0; pa < 5; ++pa)
            for (int pb = pa; pb < 5; ++pb) {
                if (!((m >> (first_pair(pa) + pb - pa)) & 1u)) continue;
                const int b = block(nd[pa], nd[pb]);
                CHECK(b >= 0, "%s: pair outside the pattern", name);
                const uint32_t grad = pa == pb ? (uint32_t)(total - 32u + 6u * pa) : 0xffffffffu;
                expect[b].push_back({(uint32_t)(L.off[g] + 36u * rank), grad});
                ++rank;
            }
    }
    CHECK(L.total == total && L.off[nseg] == total, "%s: total", name);
    CHECK((int)L.ent_ptr.size() == nb + 1 && L.ent_ptr[0] == 0, "%s: ent_ptr size", name);
    size_t nent = 0;
    for (int b = 0; b < nb && failures == 0; ++b) {
        const auto& e = expect[b];
        nent += e.size();
        CHECK(L.ent_ptr[b + 1] - L.ent_ptr[b] == (int)e.size(), "%s: block %d entry count", name, b);
        for (size_t j = 0; j < e.size() && failures == 0; ++j) {
            CHECK(L.ent_sub[L.ent_ptr[b] + j] == e[j].first, "%s: block %d entry %zu sub", name, b, j);
            CHECK(L.ent_grad[L.ent_ptr[b] + j] == e[j].second, "%s: block %d entry %zu grad", name, b, j);
        }
    }
    CHECK(L.ent_sub.size() == nent && L.ent_grad.size() == nent, "%s: entry totals", name);
    // packs: whole segments, at most max_surfels, greedy
    const int npk = (int)L.pack_start.size() - 1;
    CHECK(npk >= 1 && L.pack_seg.size() == L.pack_start.size(), "%s: pack sizes", name);
    CHECK(L.pack_start.back() == ns && L.pack_seg.back() == nseg && L.pack_seg[0] == 0, "%s: packs cover", name);
    for (int k = 0; k < npk; ++k) {
        const int g0 = L.pack_seg[k], g1 = L.pack_seg[k + 1];
        CHECK(g1 > g0, "%s: empty pack %d", name, k);
        CHECK(L.pack_start[k] == L.seg_start[g0] && L.pack_start[k + 1] == L.seg_start[g1], "%s: pack %d bounds", name, k);
        CHECK(L.pack_start[k + 1] - L.pack_start[k] <= max_surfels, "%s: pack %d too long", name, k);
        if (g1 < nseg)
            CHECK(L.seg_start[g1 + 1] - L.pack_start[k] > max_surfels, "%s: pack %d ends early", name, k);
    }
}

static void run(const char* name, int nn, const std::vector<std::vector<int>>& sets, int max_surfels,
                std::mt19937& rng) {
    Problem P = make_problem(nn, sets, rng);
    SegmentLayout L;
    std::string why;
    const bool ok = swgn::segment_layout((int)P.key.size(), nn, (int)P.col_idx.size(), P.key.data(), P.idx4.data(),
                                         P.row_ptr.data(), P.col_idx.data(), max_surfels, L, why);
    CHECK(ok, "%s: segment_layout failed: %s", name, why.c_str());
    if (ok) verify(P, max_surfels, L, name);
    printf("%s: ns=%zu segments=%zu packs=%zu entries=%zu floats=%llu\n", name, P.key.size(), L.mask.size(),
           L.pack_start.size() - 1, L.ent_sub.size(), (unsigned long long)L.total);
}

static std::vector<int> four_near(int nn, int window, std::mt19937& rng) {
    // 4 distinct nodes in [base, base + window), window >= 4
    std::uniform_int_distribution<int> c(0, nn - window), d(0, window - 1);
    const int base = c(rng);
    std::set<int> s;
    while (s.size() < 4) s.insert(base + d(rng));
    return std::vector<int>(s.begin(), s.end());
}

int main() {
    std::mt19937 rng(1904);
    // a 5-node run followed by a surfel with 4 new nodes (union of 9)
    run("disjoint_after_five", 16, {{0, 1, 2, 3}, {0, 1, 2, 4}, {5, 6, 7, 8}, {5, 6, 7, 9}, {10, 11, 12, 13}}, 256, rng);
    // one surfel
    run("single", 9, {{2, 4, 6, 8}}, 256, rng);
    // one node set repeated past the length cap
    run("long_run", 9, std::vector<std::vector<int>>(1000, {1, 3, 5, 7}), 256, rng);
    // the length cap at 1 and 3 surfels
    run("cap1", 12, {{0, 1, 2, 3}, {0, 1, 2, 3}, {0, 1, 2, 4}}, 1, rng);
    run("cap3", 40, [&] {
        std::vector<std::vector<int>> v;
        for (int i = 0; i < 200; ++i) v.push_back(four_near(40, 6, rng));
        return v;
    }(), 3, rng);
    // random node sets: local (mostly mergeable) and spread (rarely)
    for (int rep = 0; rep < 3; ++rep) {
        for (int window : {5, 7, 12, 64}) {
            std::vector<std::vector<int>> v;
            const int nn = 300 + 700 * rep;
            const int ns = 20000 + 15000 * rep;
            for (int i = 0; i < ns; ++i) v.push_back(four_near(nn, window, rng));
            // long runs of one set, as neighbouring surfels share nodes
            for (int i = 0; i < ns / 4; ++i) v.push_back(v[i % 97]);
            char name[64];
            snprintf(name, sizeof name, "random_nn%d_w%d", nn, window);
            run(name, nn, v, 256, rng);
        }
    }
    // rejected inputs
    {
        Problem P = make_problem(9, {{0, 1, 2, 3}, {0, 1, 2, 4}}, rng);
        SegmentLayout L;
        std::string why;
        std::vector<int32_t> bad = P.idx4;
        bad[5] = 8;   // slot node outside the node set
        CHECK(!swgn::segment_layout(2, 9, (int)P.col_idx.size(), P.key.data(), bad.data(), P.row_ptr.data(),
                                    P.col_idx.data(), 256, L, why), "accepted a slot node outside its set");
        std::vector<uint64_t> rev = {P.key[1], P.key[0]};
        CHECK(!swgn::segment_layout(2, 9, (int)P.col_idx.size(), rev.data(), P.idx4.data(), P.row_ptr.data(),
                                    P.col_idx.data(), 256, L, why), "accepted unsorted keys");
        int dup[4] = {0, 1, 1, 3};
        std::vector<uint64_t> dk = {pack4(dup), P.key[1]};
        CHECK(!swgn::segment_layout(2, 9, (int)P.col_idx.size(), dk.data(), P.idx4.data(), P.row_ptr.data(),
                                    P.col_idx.data(), 256, L, why), "accepted a repeated node");
        std::vector<int> rp(10, 0);   // empty pattern rows
        for (int i = 0; i <= 9; ++i) rp[i] = std::min(i, 9);
        std::vector<int> ci(9);
        for (int i = 0; i < 9; ++i) ci[i] = i;
        CHECK(!swgn::segment_layout(2, 9, 9, P.key.data(), P.idx4.data(), rp.data(), ci.data(), 256, L, why),
              "accepted a pattern without the node pairs");
    }
    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
