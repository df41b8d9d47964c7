// Runs the GPU library's host-side logic with no device present, for a
// build of its host code with AddressSanitizer and UndefinedBehaviorSanitizer:
// motif and partial-order checks, tree planning and candidates, the exact
// standard error, batch options, error strings and the argument checks that
// precede any device call.  Exits non-zero on any unexpected return code.
#include <cstdio>
#include <cstring>
#include <vector>

#include "timest.h"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64() {
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return rng_state;
}

#define CHECK(c)                                                                \
    do {                                                                        \
        if (!(c)) {                                                             \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                                           \
        }                                                                       \
    } while (0)

static tm_motif motif(const int (*e)[2], int l, int64_t delta) {
    tm_motif mo;
    std::memset(&mo, 0, sizeof mo);
    int k = 0;
    for (int p = 0; p < l; ++p) {
        mo.src[p] = e[p][0];
        mo.dst[p] = e[p][1];
        if (e[p][0] + 1 > k) k = e[p][0] + 1;
        if (e[p][1] + 1 > k) k = e[p][1] + 1;
    }
    mo.k = k;
    mo.l = l;
    mo.delta = delta;
    return mo;
}

int main() {
    for (int c = 0; c >= -12; --c) CHECK(tm_strerror(c) != nullptr);
    const int cyc4[4][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}};
    const int sg[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 4}, {2, 4}, {3, 4}};
    const int chain[5][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 4}, {4, 5}};
    const int star7[7][2] = {{0, 1}, {0, 2}, {0, 3}, {0, 4}, {0, 5}, {0, 6}, {0, 7}};
    const int many[16][2] = {{0, 1}, {1, 0}, {0, 1}, {1, 0}, {0, 1}, {1, 0}, {0, 1}, {1, 0},
                             {0, 1}, {1, 0}, {0, 1}, {1, 0}, {0, 1}, {1, 0}, {0, 1}, {1, 0}};
    std::vector<tm_motif> ok = {motif(cyc4, 4, 10), motif(sg, 6, 10), motif(chain, 5, 10), motif(star7, 7, 10),
                                motif(many, 16, 10)};
    // partial orders: unordered fan-out, a diamond, chains written pairwise
    tm_motif po = motif(sg, 6, 10);
    po.partial = 1;
    po.before[3] = 1u << 0;
    po.before[4] = 1u << 1;
    po.before[5] = 1u << 2;
    ok.push_back(po);
    tm_motif chain_po = motif(chain, 5, 10);
    chain_po.partial = 1;
    for (int q = 1; q < 5; ++q) chain_po.before[q] = (uint16_t)(1u << (q - 1));
    ok.push_back(chain_po);
    for (const tm_motif& mo : ok) {
        tm_tree t;
        CHECK(tm_default_tree(&mo, &t) == TM_OK);
        int n = 0;
        CHECK(tm_tree_candidates(&mo, nullptr, nullptr, 0, &n) == TM_OK && n > 0);
        std::vector<tm_tree> trees(n);
        std::vector<int64_t> loose(n);
        CHECK(tm_tree_candidates(&mo, trees.data(), loose.data(), n, &n) == TM_OK);
    }
    // malformed motifs and orders
    tm_motif bad = motif(cyc4, 4, 0);
    tm_tree t;
    CHECK(tm_default_tree(&bad, &t) == TM_EINVAL);
    bad = motif(cyc4, 4, 10);
    bad.partial = 2;
    CHECK(tm_default_tree(&bad, &t) == TM_EINVAL);
    bad.partial = 1;
    bad.before[0] = 2;  // edge 1 before edge 0: against the listing order
    CHECK(tm_default_tree(&bad, &t) == TM_EINVAL);
    tm_motif par = motif(many, 3, 10);
    par.partial = 1;  // parallel edges 0 and 2 unordered
    CHECK(tm_default_tree(&par, &t) == TM_EINVAL);
    tm_motif wide_po = motif(many, 16, 10);
    wide_po.partial = 1;  // 15 non-tree edges unordered: beyond the GPU's counter
    for (int q = 2; q < 16; ++q) wide_po.before[q] = (uint16_t)(1u << (q - 2));
    CHECK(tm_default_tree(&wide_po, &t) == TM_EINVAL);
    CHECK(tm_last_error() != nullptr);
    // the standard error on random exact sums
    for (int x = 0; x < 5000; ++x) {
        tm_result r;
        std::memset(&r, 0, sizeof r);
        r.W = {next_u64(), next_u64() >> (next_u64() % 64)};
        r.acc2 = {next_u64(), next_u64() >> 2};
        r.acc2_sq = {~0ull, ~0ull};
        r.k = next_u64() % 3 == 0 ? 1 : 2 + next_u64() % 100000000;
        r.flags = next_u64() % 5 == 0 ? TM_F_SQ_SATURATED : 0;
        CHECK(tm_result_finish(&r) == TM_OK);
    }
    CHECK(tm_result_finish(nullptr) == TM_EINVAL);
    // batch options
    tm_batch_opts prev, o = {2048, 0, 4096, 0, 1000};
    CHECK(tm_batch_options(&o, &prev) == TM_OK);
    CHECK(tm_batch_options(&prev, nullptr) == TM_OK);
    o.root_lds = 1 << 20;
    CHECK(tm_batch_options(&o, nullptr) == TM_EINVAL);
    int pt = 0, pb = 0;
    CHECK(tm_batch_config(100, 0, &pt, &pb) == TM_EINVAL);
    // argument checks before any device work
    tm_graph* g = nullptr;
    CHECK(tm_graph_create(nullptr, nullptr, nullptr, 5, 3, TM_PTR_HOST, nullptr, nullptr, &g) == TM_EINVAL);
    CHECK(tm_graph_create(nullptr, nullptr, nullptr, -1, 3, TM_PTR_HOST, nullptr, nullptr, &g) == TM_EINVAL);
    tm_allocator half = {nullptr, nullptr, nullptr};
    int32_t s[1] = {0}, d[1] = {1};
    int64_t tt[1] = {0};
    CHECK(tm_graph_create(s, d, tt, 1, 2, TM_PTR_HOST, &half, nullptr, &g) == TM_EINVAL);
    CHECK(tm_graph_create(s, d, tt, 1, 2, 7, nullptr, nullptr, &g) == TM_EINVAL);
    tm_server_opts so = {100, 1000, 0, 0};  // chunk above the pass size
    tm_server* srv = nullptr;
    CHECK(tm_server_create(1 << 30, &so, nullptr, &srv) == TM_EINVAL);
    CHECK(tm_server_create(1 << 30, nullptr, &half, &srv) == TM_EINVAL);
    tm_result r;
    CHECK(tm_sample(nullptr, 1, 0, 1, 1, nullptr, &r, nullptr) == TM_EINVAL);
    CHECK(tm_sample_noalloc(nullptr, 1, 0, 1, 1, nullptr, &r, nullptr) == TM_EINVAL);
    std::printf("host driver ok\n");
    return 0;
}
