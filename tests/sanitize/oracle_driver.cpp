// Runs the oracle's functions on small seeded graphs so that a build with
// AddressSanitizer and UndefinedBehaviorSanitizer sees every code path:
// graph building and its errors, weights under every constraint mode and
// every spanning tree, sampling, validation and completion counting (total
// and partial orders), listing, tree choice, brute force and the standard
// error on wide sums.  Exits non-zero on any unexpected return code.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "timest_oracle.h"

static uint64_t rng_state = 88172645463325252ull;
static uint64_t next_u64() {
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return rng_state;
}

static or_motif motif(const int (*e)[2], int l, int64_t delta, const int (*before)[2] = nullptr, int nb = -1) {
    or_motif mo = {};
    int k = 0;
    for (int p = 0; p < l; ++p) {
        mo.src[p] = e[p][0];
        mo.dst[p] = e[p][1];
        k = std::max(k, std::max(e[p][0], e[p][1]) + 1);
    }
    mo.k = k;
    mo.l = l;
    mo.delta = delta;
    if (nb >= 0) {
        mo.partial = 1;
        for (int x = 0; x < nb; ++x) mo.before[before[x][1]] |= (uint16_t)(1u << before[x][0]);
    }
    return mo;
}

#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                                 \
        }                                                             \
    } while (0)

int main() {
    const int m = 400, n = 12;
    std::vector<int32_t> s(m), d(m);
    std::vector<int64_t> t(m);
    for (int i = 0; i < m; ++i) {
        s[i] = (int32_t)(next_u64() % n);
        do d[i] = (int32_t)(next_u64() % n); while (d[i] == s[i]);
        t[i] = (int64_t)(next_u64() % 2000) + 1000000;
    }
    // duplicates removed by nudging times
    for (int i = 0; i < m; ++i) t[i] += i % 7;
    or_graph* g = nullptr;
    int rc = or_graph_create(s.data(), d.data(), t.data(), m, n, &g);
    if (rc == OR_EDUP) {
        for (int i = 0; i < m; ++i) t[i] = 1000000 + 5 * i + (int64_t)(next_u64() % 3);
        rc = or_graph_create(s.data(), d.data(), t.data(), m, n, &g);
    }
    CHECK(rc == OR_OK);
    // error paths
    {
        int32_t a[2] = {0, 1}, b[2] = {1, 1};
        int64_t tt[2] = {5, 6};
        or_graph* bad = nullptr;
        CHECK(or_graph_create(a, b, tt, 2, 3, &bad) == OR_ESELFLOOP);
        b[1] = 7;
        CHECK(or_graph_create(a, b, tt, 2, 3, &bad) == OR_EINVAL);
    }
    const int cyc3[3][2] = {{0, 1}, {1, 2}, {2, 0}};
    const int cyc4[4][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}};
    const int sg[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 4}, {2, 4}, {3, 4}};
    const int lt[5][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}, {0, 2}};
    const int po_free[4][2] = {{0, 1}, {1, 2}, {2, 0}, {0, 2}};
    const int po_b[1][2] = {{0, 1}};
    const int po_cyc_b[2][2] = {{0, 2}, {1, 2}};
    std::vector<or_motif> mos = {motif(cyc3, 3, 300), motif(cyc4, 4, 400), motif(sg, 6, 500), motif(lt, 5, 400),
                                 motif(po_free, 4, 400, po_b, 1), motif(cyc3, 3, 300, po_cyc_b, 2)};
    for (const or_motif& mo : mos) {
        int nt = 0;
        CHECK(or_tree_candidates(&mo, nullptr, nullptr, 0, &nt) == OR_OK && nt > 0);
        std::vector<or_tree> trees(nt);
        std::vector<int64_t> loose(nt);
        CHECK(or_tree_candidates(&mo, trees.data(), loose.data(), nt, &nt) == OR_OK);
        for (int x = 0; x < nt && x < 6; ++x) {
            for (uint32_t c = 0; c < 4; ++c) {
                or_prep* p = nullptr;
                CHECK(or_prepare_ex(g, &mo, &trees[x], c, &p) == OR_OK);
                or_result r;
                std::vector<or_rec> recs(500);
                CHECK(or_sample(p, 7, 0, 500, 500, &r, recs.data()) == OR_OK);
                std::vector<or_u128> w(m);
                CHECK(or_prep_weights(p, trees[x].edge[0], 0, w.data()) == OR_OK);
                std::vector<or_u128> wi(or_prep_q(p) + 1);
                or_prep_interval_weights(p, wi.data());
                for (int a = 0; a < 50; ++a) {
                    if (recs[a].status != 0) continue;
                    or_u128 mphi;
                    CHECK(or_derive_cnt(p, recs[a].eid, &mphi) == OR_OK);
                    if (!mo.partial && (mphi.lo | mphi.hi)) {
                        int32_t inst[16];
                        CHECK(or_list_instance(p, recs[a].eid, or_u128{0, 0}, inst) == OR_OK);
                    }
                }
                or_prep_destroy(p);
                if (c == 3) {
                    or_u128 W;
                    CHECK(or_brute_tree_weight_ex(g, &mo, &trees[x], c, &W) == OR_OK);
                }
            }
        }
        or_u128 C;
        CHECK(or_brute_count(g, &mo, &C) == OR_OK);
        or_tree best;
        or_u128 Ws[3];
        int ne = 0;
        CHECK(or_choose_tree(g, &mo, 3, &best, Ws, &ne) == OR_OK);
    }
    // partial-order errors
    {
        const int bad_b[1][2] = {{1, 0}};
        or_motif bad = motif(cyc3, 3, 10, bad_b, 1);
        or_prep* p = nullptr;
        CHECK(or_prepare(g, &bad, nullptr, &p) == OR_EINVAL);
    }
    // the standard error on sums up to 2^128
    for (int x = 0; x < 2000; ++x) {
        or_u128 W = {next_u64(), next_u64() >> (next_u64() % 64)};
        or_u128 s1 = {next_u64(), next_u64() >> 3};
        or_u128 s2 = {~0ull, ~0ull >> 1};
        volatile double se = or_std_error(W, s1, s2, 2 + next_u64() % 1000000, 0);
        (void)se;
    }
    or_graph_destroy(g);
    std::printf("oracle driver ok\n");
    return 0;
}
