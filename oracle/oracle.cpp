// TIMEST reference oracle -- TEST INFRASTRUCTURE ONLY (see timest_oracle.h).
//
// Plain single-threaded C++ written from the paper (arXiv 2507.20441):
// every step is the definition or the algorithm written out, with no blocking,
// fusion or reordering beyond what the paper states.  Exact integers
// (unsigned __int128) throughout; overflow is reported, never wrapped.

#include "timest_oracle.h"
#include "graph_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <utility>
#include <vector>

typedef unsigned __int128 u128;

static or_u128 to_or(u128 x) { return or_u128{(uint64_t)x, (uint64_t)(x >> 64)}; }
static u128 from_or(or_u128 x) { return ((u128)x.hi << 64) | x.lo; }

// Checked arithmetic: returns false on overflow.
static bool add_ok(u128 a, u128 b, u128* r) { *r = a + b; return *r >= a; }
static bool mul_ok(u128 a, u128 b, u128* r) { return !__builtin_mul_overflow(a, b, r); }

static const int64_t kMaxSpan = (int64_t)1 << 62;

// ------------------------------------------------------------------------
// Graph construction (container in graph_internal.h).
// ------------------------------------------------------------------------
extern "C" int or_graph_create(const int32_t* src, const int32_t* dst, const int64_t* t,
                               int64_t m, int32_t n, or_graph** out) {
    if (!out || m < 0 || n < 0 || (m > 0 && (!src || !dst || !t)) || m >= ((int64_t)1 << 31))
        return OR_EINVAL;
    // First failing check wins, in this order: id range, self loop, span, duplicate.
    for (int64_t i = 0; i < m; ++i)
        if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) return OR_EINVAL;
    for (int64_t i = 0; i < m; ++i)
        if (src[i] == dst[i]) return OR_ESELFLOOP;
    int64_t tmin = 0, tmax = 0;
    for (int64_t i = 0; i < m; ++i) {
        if (i == 0 || t[i] < tmin) tmin = t[i];
        if (i == 0 || t[i] > tmax) tmax = t[i];
    }
    if (m > 0 && ((__int128)tmax - (__int128)tmin) >= kMaxSpan) return OR_ERANGE;

    or_graph* g = new or_graph();
    g->n = n;
    g->m = m;
    g->shift = tmin;
    g->T = tmax - tmin;
    g->e.resize(m);
    for (int64_t i = 0; i < m; ++i) g->e[i] = OEdge{src[i], dst[i], t[i] - tmin};
    std::sort(g->e.begin(), g->e.end(), [](const OEdge& a, const OEdge& b) {
        if (a.t != b.t) return a.t < b.t;
        if (a.u != b.u) return a.u < b.u;
        return a.v < b.v;
    });
    // Each tuple (u,v,t) may appear only once (Sec. 1.1).
    for (int64_t i = 1; i < m; ++i) {
        const OEdge& a = g->e[i - 1];
        const OEdge& b = g->e[i];
        if (a.t == b.t && a.u == b.u && a.v == b.v) {
            delete g;
            return OR_EDUP;
        }
    }
    g->out.resize(n);
    g->in.resize(n);
    for (int64_t id = 0; id < m; ++id) {
        const OEdge& x = g->e[id];
        g->out[x.u].push_back((int32_t)id);
        g->in[x.v].push_back((int32_t)id);
        g->el[{x.u, x.v}].push_back((int32_t)id);
    }
    *out = g;
    return OR_OK;
}

extern "C" void or_graph_destroy(or_graph* g) { delete g; }

extern "C" void or_graph_edges(const or_graph* g, int32_t* src, int32_t* dst, int64_t* t) {
    for (int64_t i = 0; i < g->m; ++i) {
        if (src) src[i] = g->e[i].u;
        if (dst) dst[i] = g->e[i].v;
        if (t) t[i] = g->e[i].t;
    }
}

extern "C" int64_t or_graph_shift(const or_graph* g) { return g->shift; }

extern "C" int64_t or_graph_list(const or_graph* g, int32_t vertex, int dir, int32_t* eids,
                                 int64_t cap) {
    if (vertex < 0 || vertex >= g->n) return -1;
    const std::vector<int32_t>& L = dir > 0 ? g->out[vertex] : g->in[vertex];
    for (int64_t i = 0; i < (int64_t)L.size() && i < cap; ++i) eids[i] = L[i];
    return (int64_t)L.size();
}

// First position in an eid list (sorted by time) whose edge time is >= t0.
static size_t first_at_or_after(const or_graph& g, const std::vector<int32_t>& L, int64_t t0) {
    size_t lo = 0, hi = L.size();
    while (lo < hi) {
        size_t mid = (lo + hi) / 2;
        if (g.e[L[mid]].t < t0) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------------------
// Motif and spanning tree (Def. "temporal motif", Def. "dependency list",
// Def. "spanning tree of a temporal motif").
// ------------------------------------------------------------------------
// The time-order relation of the motif: R[q] holds edge p when p must be
// strictly earlier than q.  Total order: every p < q.  Partial order: the
// transitive closure of the given pairs (each p < q, so one pass in q order
// closes it).
static void order_relation(const or_motif* mo, uint16_t R[16]) {
    for (int q = 0; q < 16; ++q) {
        R[q] = 0;
        if (q >= mo->l) continue;
        if (!mo->partial) {
            R[q] = (uint16_t)((1u << q) - 1u);
            continue;
        }
        uint16_t r = mo->before[q];
        for (int p = 0; p < q; ++p)
            if ((mo->before[q] >> p) & 1u) r |= R[p];
        R[q] = r;
    }
}

static bool precedes(const uint16_t R[16], int p, int q) { return (R[q] >> p) & 1u; }

static bool motif_ok(const or_motif* mo) {
    if (!mo || mo->k < 2 || mo->k > 8 || mo->l < 1 || mo->l > 16) return false;
    if (mo->partial > 1) return false;
    if (mo->partial) {
        // pairs only from an earlier listed edge to a later one
        for (int q = 0; q < 16; ++q)
            if (mo->before[q] & (uint16_t)~((1u << (q < mo->l ? q : 0)) - 1u)) return false;
        uint16_t R[16];
        order_relation(mo, R);
        // parallel motif edges must be ordered: otherwise both could take the
        // same graph edge and the edge map would not be 1-1
        for (int p = 0; p < mo->l; ++p)
            for (int q = p + 1; q < mo->l; ++q)
                if (mo->src[p] == mo->src[q] && mo->dst[p] == mo->dst[q] && !precedes(R, p, q)) return false;
    }
    if (mo->delta < 1 || mo->delta >= kMaxSpan) return false;
    for (int p = 0; p < mo->l; ++p) {
        if (mo->src[p] < 0 || mo->src[p] >= mo->k || mo->dst[p] < 0 || mo->dst[p] >= mo->k) return false;
        if (mo->src[p] == mo->dst[p]) return false;
    }
    // weakly connected: every vertex reachable from vertex 0 ignoring direction
    bool seen[8] = {false};
    seen[0] = true;
    for (int pass = 0; pass < mo->k; ++pass)
        for (int p = 0; p < mo->l; ++p)
            if (seen[mo->src[p]] || seen[mo->dst[p]]) seen[mo->src[p]] = seen[mo->dst[p]] = true;
    for (int x = 0; x < mo->k; ++x)
        if (!seen[x]) return false;
    return true;
}

// A set of k-1 motif edges is a spanning tree iff adding them one by one
// never joins two already-connected vertices.
static bool is_spanning_tree(const or_motif* mo, const int32_t* edges, int cnt) {
    if (cnt != mo->k - 1) return false;
    int comp[8];
    for (int x = 0; x < mo->k; ++x) comp[x] = x;
    for (int j = 0; j < cnt; ++j) {
        int p = edges[j];
        if (p < 0 || p >= mo->l) return false;
        for (int j2 = 0; j2 < j; ++j2)
            if (edges[j2] == p) return false;
        int a = comp[mo->src[p]], b = comp[mo->dst[p]];
        if (a == b) return false;
        for (int x = 0; x < mo->k; ++x)
            if (comp[x] == b) comp[x] = a;
    }
    return true;
}

static bool tree_ok(const or_motif* mo, const or_tree* tr) {
    if (!tr || !is_spanning_tree(mo, tr->edge, tr->n_edges)) return false;
    for (int j = 0; j < tr->n_edges; ++j)
        if (tr->edge[j] == tr->center) return true;
    return false;
}

struct Plan {
    or_motif mo;
    uint16_t R[16];      // time-order relation: R[q] holds p when p is strictly earlier than q
    int center = -1;
    bool in_tree[16] = {false};
    int parent[16];
    int attach[16];      // motif vertex shared with the parent edge
    int lower[16];       // v_s: the endpoint of s further from the center
    int alpha[16];       // +1: child leaves the attach vertex; -1: enters it
    int beta[16];        // -1: child precedes its parent ('<'); +1: follows ('>'); 0: unordered
    int height[16];
    int H = 0;
    std::vector<int> children[16];
    std::vector<int> preorder;     // center first, then children subtree by subtree
    std::vector<int> tree_sorted;  // tree edges by increasing pi index
};

static void attach_children(Plan& P, int s, int z) {
    // Every tree edge other than s touching z hangs below s at z.
    for (int p = 0; p < P.mo.l; ++p) {
        if (!P.in_tree[p] || p == s || p == P.parent[s]) continue;
        if (P.mo.src[p] != z && P.mo.dst[p] != z) continue;
        if (P.parent[p] != -2) continue;  // already placed
        P.parent[p] = s;
        P.attach[p] = z;
        P.lower[p] = (P.mo.src[p] == z) ? P.mo.dst[p] : P.mo.src[p];
        P.alpha[p] = (P.mo.src[p] == z) ? +1 : -1;
        // '<' when the child must precede its parent, '>' when it must
        // follow, '~' (0) when a partial order leaves the pair unordered
        P.beta[p] = precedes(P.R, p, s) ? -1 : (precedes(P.R, s, p) ? +1 : 0);
        P.children[s].push_back(p);
        attach_children(P, p, P.lower[p]);
    }
}

static int compute_height(Plan& P, int s) {
    int h = 0;
    for (int c : P.children[s]) h = std::max(h, 1 + compute_height(P, c));
    P.height[s] = h;
    return h;
}

static void build_preorder(Plan& P, int s) {
    P.preorder.push_back(s);
    for (int c : P.children[s]) build_preorder(P, c);
}

static void make_plan(const or_motif* mo, const or_tree* tr, Plan& P) {
    P.mo = *mo;
    order_relation(mo, P.R);
    P.center = tr->center;
    for (int p = 0; p < 16; ++p) {
        P.parent[p] = -2;
        P.attach[p] = P.lower[p] = -1;
        P.alpha[p] = P.beta[p] = 0;
        P.height[p] = 0;
    }
    for (int j = 0; j < tr->n_edges; ++j) P.in_tree[tr->edge[j]] = true;
    int c = tr->center;
    P.parent[c] = -1;
    attach_children(P, c, mo->src[c]);
    attach_children(P, c, mo->dst[c]);
    for (int p = 0; p < 16; ++p) std::sort(P.children[p].begin(), P.children[p].end());
    P.H = compute_height(P, c);
    build_preorder(P, c);
    for (int p = 0; p < mo->l; ++p)
        if (P.in_tree[p]) P.tree_sorted.push_back(p);
}

// Default tree: the spanning tree with the smallest constraint looseness
// (Alg. 8, read per tree vertex over pairs of incident tree edges as
// |pi(e1) - pi(e2)| - 1), ties to the lexicographically smallest edge set;
// center: the tree edge giving the smallest rooted height, ties to the
// smallest pi index.
extern "C" int or_default_tree(const or_motif* mo, or_tree* out) {
    if (!motif_ok(mo) || !out) return OR_EINVAL;
    int need = mo->k - 1;
    long best = -1;
    int best_set[8] = {0};
    int cur[8];
    // enumerate subsets of size need in lexicographic order
    std::vector<int> idx(need);
    for (int j = 0; j < need; ++j) idx[j] = j;
    while (true) {
        for (int j = 0; j < need; ++j) cur[j] = idx[j];
        if (is_spanning_tree(mo, cur, need)) {
            long loose = 0;
            for (int x = 0; x < mo->k; ++x)
                for (int a = 0; a < need; ++a)
                    for (int b = a + 1; b < need; ++b) {
                        int pa = cur[a], pb = cur[b];
                        bool ia = mo->src[pa] == x || mo->dst[pa] == x;
                        bool ib = mo->src[pb] == x || mo->dst[pb] == x;
                        if (ia && ib) loose += std::abs(pa - pb) - 1;
                    }
            if (best < 0 || loose < best) {
                best = loose;
                for (int j = 0; j < need; ++j) best_set[j] = cur[j];
            }
        }
        int j = need - 1;
        while (j >= 0 && idx[j] == mo->l - need + j) --j;
        if (j < 0) break;
        ++idx[j];
        for (int j2 = j + 1; j2 < need; ++j2) idx[j2] = idx[j2 - 1] + 1;
    }
    if (best < 0) return OR_EINVAL;
    or_tree t;
    std::memset(&t, 0, sizeof t);
    t.n_edges = need;
    for (int j = 0; j < need; ++j) t.edge[j] = best_set[j];
    int best_h = 1 << 30;
    for (int j = 0; j < need; ++j) {
        t.center = best_set[j];
        Plan P;
        make_plan(mo, &t, P);
        if (P.H < best_h) {
            best_h = P.H;
            out->center = best_set[j];
        }
    }
    out->n_edges = need;
    for (int j = 0; j < 8; ++j) out->edge[j] = j < need ? best_set[j] : 0;
    return OR_OK;
}

// ------------------------------------------------------------------------
// Alg. 8 (constraint looseness) and Alg. 7 (choose the tree by W).
// ------------------------------------------------------------------------
struct OCand {
    long loose;
    std::vector<int> edges;
    int height;
    int center;
};

// Every spanning tree (edge subsets of size k-1 that connect the motif), each
// with every choice of center.
static std::vector<OCand> all_candidates(const or_motif* mo) {
    std::vector<OCand> out;
    const int need = mo->k - 1;
    std::vector<int> idx(need);
    for (int j = 0; j < need; ++j) idx[j] = j;
    while (need > 0) {
        int cur[8];
        for (int j = 0; j < need; ++j) cur[j] = idx[j];
        if (is_spanning_tree(mo, cur, need)) {
            // Alg. 8 (reading: over the tree's own edges): for every vertex,
            // every unordered pair of tree edges on it adds |pi(e1) - pi(e2)| - 1
            long loose = 0;
            for (int x = 0; x < mo->k; ++x)
                for (int a = 0; a < need; ++a)
                    for (int b = a + 1; b < need; ++b) {
                        const bool ia = mo->src[cur[a]] == x || mo->dst[cur[a]] == x;
                        const bool ib = mo->src[cur[b]] == x || mo->dst[cur[b]] == x;
                        if (ia && ib) loose += std::abs(cur[a] - cur[b]) - 1;
                    }
            for (int j = 0; j < need; ++j) {
                or_tree t;
                std::memset(&t, 0, sizeof t);
                t.n_edges = need;
                for (int x = 0; x < need; ++x) t.edge[x] = cur[x];
                t.center = cur[j];
                Plan P;
                make_plan(mo, &t, P);
                out.push_back(OCand{loose, std::vector<int>(cur, cur + need), P.H, cur[j]});
            }
        }
        int j = need - 1;
        while (j >= 0 && idx[j] == mo->l - need + j) --j;
        if (j < 0) break;
        ++idx[j];
        for (int j2 = j + 1; j2 < need; ++j2) idx[j2] = idx[j2 - 1] + 1;
    }
    std::stable_sort(out.begin(), out.end(), [](const OCand& a, const OCand& b) {
        if (a.loose != b.loose) return a.loose < b.loose;
        if (a.edges != b.edges) return a.edges < b.edges;
        if (a.height != b.height) return a.height < b.height;
        return a.center < b.center;
    });
    return out;
}

static or_tree cand_tree(const OCand& c) {
    or_tree t;
    std::memset(&t, 0, sizeof t);
    t.n_edges = (int32_t)c.edges.size();
    for (size_t x = 0; x < c.edges.size(); ++x) t.edge[x] = c.edges[x];
    t.center = c.center;
    return t;
}

extern "C" int or_tree_candidates(const or_motif* mo, or_tree* out, int64_t* looseness, int max_out,
                                  int* n_out) {
    if (!motif_ok(mo) || !n_out) return OR_EINVAL;
    const std::vector<OCand> c = all_candidates(mo);
    *n_out = (int)c.size();
    for (int x = 0; x < max_out && x < (int)c.size(); ++x) {
        out[x] = cand_tree(c[x]);
        if (looseness) looseness[x] = c[x].loose;
    }
    return OR_OK;
}

// ------------------------------------------------------------------------
// Preprocessing: Alg. 1 (intervals) and Alg. 2 (bottom-up s-weights).
// ------------------------------------------------------------------------
struct or_prep {
    const or_graph* g = nullptr;
    Plan P;
    int64_t delta = 0;
    int64_t q = 0;
    std::vector<int64_t> lo, hi;       // eid range of G_i: edges with t in I_i
    std::vector<int64_t> base;         // offset of G_i's block in the weight tables
    std::vector<u128> w[16];           // w_i(s,e) at base[i] + (e - lo[i]); non-leaf s only
    std::vector<u128> Wi;              // W_i
    std::vector<u128> cumW;            // cumW[i] = sum_{i'<i} W_i', q+1 entries
    std::vector<std::vector<u128>> root_cum;  // per interval: prefix of w_i(c,e) over G_i
    u128 W = 0;
    // constraints (Sec. "A Closer Look at Preprocessing"): constraint 1 (order
    // and delta between a tree edge and its parent) always; constraint 2
    // (distinct end vertices of adjacent edges) when flags has OR_C_EXCLUDE;
    // constraint 3 (the 2 delta intervals) when it has OR_C_WINDOWS, else a
    // single interval over the whole span
    uint32_t flags = OR_C_ALL;
    int64_t ilen = 0;  // interval unit: delta, or T + 1 without constraint 3
};

static bool in_interval(int64_t t, int64_t i, int64_t delta) {
    return t >= i * delta && t < (i + 2) * delta;
}

// s-weight lookup: a leaf edge has weight 1 (Alg. 2 skips height 0).
static u128 weight(const or_prep& R, int64_t i, int s, int32_t e) {
    if (R.P.children[s].empty()) return 1;
    return R.w[s][R.base[i] + (e - R.lo[i])];
}

// Candidate matches for child c of tree edge s, when s is matched to edge e
// inside G_i (Claim "matching-edges-set"): the edges at the image g of the
// attach vertex, leaving it (alpha=+) or entering it (alpha=-), whose time lies
// in [t-delta, t] (beta '<') or [t, t+delta] (beta '>') -- or, for a pair a
// partial order leaves unordered, in [t-delta, t+delta] -- that lie in G_i,
// and whose far endpoint is not the image o of s's other endpoint.  In eid
// order.
static void candidates(const or_prep& R, int64_t i, int s, int32_t e, int c,
                       std::vector<int32_t>& cand) {
    const or_graph& G = *R.g;
    const Plan& P = R.P;
    const OEdge& E = G.e[e];
    int32_t g = (P.attach[c] == P.mo.src[s]) ? E.u : E.v;
    int32_t o = (P.attach[c] == P.mo.src[s]) ? E.v : E.u;
    int64_t wlo = P.beta[c] > 0 ? E.t : E.t - R.delta;
    int64_t whi = P.beta[c] < 0 ? E.t : E.t + R.delta;
    const std::vector<int32_t>& L = P.alpha[c] > 0 ? G.out[g] : G.in[g];
    cand.clear();
    for (size_t x = first_at_or_after(G, L, wlo); x < L.size(); ++x) {
        const OEdge& F = G.e[L[x]];
        if (F.t > whi) break;
        if (!in_interval(F.t, i, R.ilen)) continue;
        int32_t far = P.alpha[c] > 0 ? F.v : F.u;
        if ((R.flags & OR_C_EXCLUDE) && far == o) continue;
        cand.push_back(L[x]);
    }
}

extern "C" int or_prepare(const or_graph* g, const or_motif* mo, const or_tree* tr, or_prep** out) {
    return or_prepare_ex(g, mo, tr, OR_C_ALL, out);
}

extern "C" int or_prepare_ex(const or_graph* g, const or_motif* mo, const or_tree* tr, uint32_t flags,
                             or_prep** out) {
    if (!g || !out || !motif_ok(mo) || (flags & ~(uint32_t)OR_C_ALL)) return OR_EINVAL;
    or_tree def;
    if (!tr) {
        if (or_default_tree(mo, &def) != OR_OK) return OR_EINVAL;
        tr = &def;
    }
    if (!tree_ok(mo, tr)) return OR_EINVAL;
    or_prep* R = new or_prep();
    R->g = g;
    make_plan(mo, tr, R->P);
    R->delta = mo->delta;
    R->flags = flags;
    R->ilen = (flags & OR_C_WINDOWS) ? mo->delta : g->T + 1;
    const int64_t d = R->ilen;
    // Alg. 1: q overlapping 2*delta intervals cover every match.
    R->q = g->m > 0 ? g->T / d + 1 : 0;
    R->lo.resize(R->q);
    R->hi.resize(R->q);
    R->base.resize(R->q + 1);
    R->base[0] = 0;
    for (int64_t i = 0; i < R->q; ++i) {
        int64_t a = 0, b = g->m;  // first eid with t >= i*d
        while (a < b) { int64_t mid = (a + b) / 2; if (g->e[mid].t < i * d) a = mid + 1; else b = mid; }
        R->lo[i] = a;
        b = g->m;                 // first eid with t >= (i+2)*d
        while (a < b) { int64_t mid = (a + b) / 2; if (g->e[mid].t < (i + 2) * d) a = mid + 1; else b = mid; }
        R->hi[i] = a;
        R->base[i + 1] = R->base[i] + (R->hi[i] - R->lo[i]);
    }
    const Plan& P = R->P;
    for (int p = 0; p < mo->l; ++p)
        if (P.in_tree[p] && !P.children[p].empty()) R->w[p].assign(R->base[R->q], 0);

    std::vector<int32_t> cand;
    R->Wi.assign(R->q, 0);
    for (int64_t i = 0; i < R->q; ++i) {                 // Alg. 1: each subgraph G_i
        for (int h = 1; h <= P.H; ++h) {                 // Alg. 2: heights bottom-up
            for (int64_t e = R->lo[i]; e < R->hi[i]; ++e) {
                for (int s = 0; s < mo->l; ++s) {
                    if (!P.in_tree[s] || P.height[s] != h) continue;
                    // Claim "overall-num-matches": product over the dependency
                    // list of the summed child weights over the candidate list.
                    u128 prod = 1;
                    for (int c : P.children[s]) {
                        candidates(*R, i, s, (int32_t)e, c, cand);
                        u128 sum = 0;
                        for (int32_t f : cand)
                            if (!add_ok(sum, weight(*R, i, c, f), &sum)) { delete R; return OR_EOVERFLOW; }
                        if (!mul_ok(prod, sum, &prod)) { delete R; return OR_EOVERFLOW; }
                    }
                    R->w[s][R->base[i] + (e - R->lo[i])] = prod;
                }
            }
        }
        // Claim "num-matches-entire-tree": W_i sums the center weights.
        u128 Wi = 0;
        for (int64_t e = R->lo[i]; e < R->hi[i]; ++e)
            if (!add_ok(Wi, weight(*R, i, P.center, (int32_t)e), &Wi)) { delete R; return OR_EOVERFLOW; }
        R->Wi[i] = Wi;
    }
    R->cumW.assign(R->q + 1, 0);
    for (int64_t i = 0; i < R->q; ++i)
        if (!add_ok(R->cumW[i], R->Wi[i], &R->cumW[i + 1])) { delete R; return OR_EOVERFLOW; }
    R->W = R->cumW[R->q];
    R->root_cum.resize(R->q);
    for (int64_t i = 0; i < R->q; ++i) {
        std::vector<u128>& rc = R->root_cum[i];
        rc.assign(R->hi[i] - R->lo[i] + 1, 0);
        for (int64_t e = R->lo[i]; e < R->hi[i]; ++e)
            rc[e - R->lo[i] + 1] = rc[e - R->lo[i]] + weight(*R, i, P.center, (int32_t)e);
    }
    *out = R;
    return OR_OK;
}

extern "C" int or_prepare_light(const or_graph* g, const or_motif* mo, const or_tree* tr, or_prep** out) {
    return or_prepare_light_ex(g, mo, tr, OR_C_ALL, out);
}

extern "C" int or_prepare_light_ex(const or_graph* g, const or_motif* mo, const or_tree* tr, uint32_t flags,
                                   or_prep** out) {
    if (!g || !out || !motif_ok(mo) || (flags & ~(uint32_t)OR_C_ALL)) return OR_EINVAL;
    or_tree def;
    if (!tr) {
        if (or_default_tree(mo, &def) != OR_OK) return OR_EINVAL;
        tr = &def;
    }
    if (!tree_ok(mo, tr)) return OR_EINVAL;
    or_prep* R = new or_prep();
    R->g = g;
    make_plan(mo, tr, R->P);
    R->delta = mo->delta;
    R->flags = flags;
    R->ilen = (flags & OR_C_WINDOWS) ? mo->delta : g->T + 1;
    R->q = g->m > 0 ? g->T / R->ilen + 1 : 0;
    *out = R;
    return OR_OK;
}

// Claim "overall-num-matches" for one edge: the product over s's children of
// the summed child weights over the candidate list, each child weight again
// by this rule (a leaf has weight 1).
static int lazy_weight(const or_prep& R, int64_t i, int s, int32_t e, uint64_t& budget, u128* out) {
    const Plan& P = R.P;
    if (P.children[s].empty()) {
        *out = 1;
        return OR_OK;
    }
    u128 prod = 1;
    std::vector<int32_t> cand;
    for (int c : P.children[s]) {
        candidates(R, i, s, e, c, cand);
        if (cand.size() > budget) return OR_ERANGE;
        budget -= cand.size();
        const std::vector<int32_t> mine(cand);
        u128 sum = 0;
        for (int32_t f : mine) {
            u128 x;
            const int rc = lazy_weight(R, i, c, f, budget, &x);
            if (rc != OR_OK) return rc;
            if (!add_ok(sum, x, &sum)) return OR_EOVERFLOW;
        }
        if (!mul_ok(prod, sum, &prod)) return OR_EOVERFLOW;
    }
    *out = prod;
    return OR_OK;
}

extern "C" int or_edge_weight(const or_prep* p, int64_t interval, int32_t s, int32_t eid, uint64_t work_limit,
                              or_u128* w) {
    if (!p || !w || eid < 0 || eid >= p->g->m || interval < 0 || interval >= p->q) return OR_EINVAL;
    if (s < 0 || s >= p->P.mo.l || !p->P.in_tree[s]) return OR_EINVAL;
    if (!in_interval(p->g->e[eid].t, interval, p->ilen)) return OR_EINVAL;
    uint64_t budget = work_limit;
    u128 x;
    const int rc = lazy_weight(*p, interval, s, eid, budget, &x);
    if (rc != OR_OK) return rc;
    *w = to_or(x);
    return OR_OK;
}

extern "C" void or_prep_destroy(or_prep* p) { delete p; }

// Alg. 7: W of the first n_c candidates (full preprocessing each); the
// smallest W wins, the earlier candidate among equals.
extern "C" int or_choose_tree(const or_graph* g, const or_motif* mo, int n_c, or_tree* best, or_u128* W_out,
                              int* n_eval) {
    if (!g || !best || n_c < 1 || !motif_ok(mo)) return OR_EINVAL;
    const std::vector<OCand> c = all_candidates(mo);
    const int n = std::min<int>(n_c, (int)c.size());
    int arg = -1;
    u128 bestW = 0;
    for (int x = 0; x < n; ++x) {
        const or_tree t = cand_tree(c[x]);
        or_prep* p = nullptr;
        const int rc = or_prepare(g, mo, &t, &p);
        if (rc != OR_OK) return rc;
        const u128 W = p->W;
        or_prep_destroy(p);
        if (W_out) W_out[x] = to_or(W);
        if (arg < 0 || W < bestW) {
            arg = x;
            bestW = W;
        }
    }
    *best = cand_tree(c[arg]);
    if (n_eval) *n_eval = n;
    return OR_OK;
}
extern "C" or_u128 or_prep_W(const or_prep* p) { return to_or(p->W); }
extern "C" int64_t or_prep_q(const or_prep* p) { return p->q; }

extern "C" void or_prep_interval_weights(const or_prep* p, or_u128* wi) {
    for (int64_t i = 0; i < p->q; ++i) wi[i] = to_or(p->Wi[i]);
}

extern "C" int or_prep_weights(const or_prep* p, int32_t s, int slot, or_u128* out) {
    if (s < 0 || s >= p->P.mo.l || !p->P.in_tree[s] || slot < 0 || slot > 1) return OR_EINVAL;
    const or_graph& G = *p->g;
    for (int64_t e = 0; e < G.m; ++e) {
        int64_t i = G.e[e].t / p->ilen - slot;
        if (i < 0 || i >= p->q) { out[e] = to_or(0); continue; }
        out[e] = to_or(weight(*p, i, s, (int32_t)e));
    }
    return OR_OK;
}

// ------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// multiply-xor S-box on a 4x32 counter with a 2x32 key bumped by the Weyl
// constants between rounds.
// ------------------------------------------------------------------------
extern "C" void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// floor(X * n / 2^128) by schoolbook multiplication in 64-bit limbs.
static u128 scale_to_range(u128 X, u128 n) {
    uint64_t x0 = (uint64_t)X, x1 = (uint64_t)(X >> 64);
    uint64_t n0 = (uint64_t)n, n1 = (uint64_t)(n >> 64);
    u128 p00 = (u128)x0 * n0, p01 = (u128)x0 * n1, p10 = (u128)x1 * n0, p11 = (u128)x1 * n1;
    u128 mid = (p00 >> 64) + (uint64_t)p01 + (uint64_t)p10;
    return p11 + (p01 >> 64) + (p10 >> 64) + (mid >> 64);
}

static u128 draw(uint64_t seed, uint64_t j, uint32_t d, u128 n) {
    uint32_t ctr[4] = {(uint32_t)j, (uint32_t)(j >> 32), d, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    or_philox4x32_10(ctr, key, x);
    u128 X = (u128)x[0] | ((u128)x[1] << 32) | ((u128)x[2] << 64) | ((u128)x[3] << 96);
    return scale_to_range(X, n);
}

extern "C" or_u128 or_draw(uint64_t seed, uint64_t j, uint32_t d, or_u128 n) {
    return to_or(draw(seed, j, d, from_or(n)));
}

// ------------------------------------------------------------------------
// Alg. 4 (ValidateAndDeriveCnt) and Alg. 5 (DeriveCnt).
// ------------------------------------------------------------------------

// ListCount: number of chains (x_1, ..., x_r), x_j in lists[j], with
// after < t(x_1) < t(x_2) < ... < t(x_r) <= upto.  Dynamic programming over the
// lists with a pointer traversal: cnt_j(x) = sum of cnt_{j-1}(y) over y with
// t(y) < t(x).  Returns false on overflow.
static bool list_count(const or_graph& G, const std::vector<std::vector<int32_t>>& lists,
                       size_t first, int64_t after, int64_t upto, u128* result) {
    if (first == lists.size()) { *result = 1; return true; }
    std::vector<int64_t> pt, ct;
    std::vector<u128> pc, cc;
    for (size_t j = first; j < lists.size(); ++j) {
        ct.clear();
        cc.clear();
        for (int32_t x : lists[j]) {
            int64_t tx = G.e[x].t;
            if (tx > after && tx <= upto) ct.push_back(tx);
        }
        cc.assign(ct.size(), 0);
        if (j == first) {
            for (size_t a = 0; a < ct.size(); ++a) cc[a] = 1;
        } else {
            u128 acc = 0;
            size_t y = 0;
            for (size_t a = 0; a < ct.size(); ++a) {
                while (y < pt.size() && pt[y] < ct[a]) {
                    if (!add_ok(acc, pc[y], &acc)) return false;
                    ++y;
                }
                cc[a] = acc;
            }
        }
        pt.swap(ct);
        pc.swap(cc);
    }
    u128 total = 0;
    for (u128 v : pc)
        if (!add_ok(total, v, &total)) return false;
    *result = total;
    return true;
}

// Completions under a partial order: one edge per list, lists in motif
// order, each choice checked against the edges chosen before it (the
// relation's pairs and distinctness); the delta range once all are chosen.
static bool po_enumerate(const or_graph& G, const or_motif& M, const uint16_t R[16],
                         const std::vector<std::vector<int32_t>>& lists, int p, std::vector<int32_t>& pick,
                         u128* count) {
    if (p == M.l) {
        int64_t lo = G.e[pick[0]].t, hi = lo;
        for (int q = 1; q < M.l; ++q) {
            lo = std::min(lo, G.e[pick[q]].t);
            hi = std::max(hi, G.e[pick[q]].t);
        }
        if (hi - lo <= M.delta) return add_ok(*count, 1, count);
        return true;
    }
    for (int32_t x : lists[p]) {
        bool ok = true;
        for (int q = 0; q < p && ok; ++q) {
            if (pick[q] == x) ok = false;
            if (precedes(R, q, p) && !(G.e[pick[q]].t < G.e[x].t)) ok = false;
        }
        if (!ok) continue;
        pick[p] = x;
        if (!po_enumerate(G, M, R, lists, p + 1, pick, count)) return false;
    }
    return true;
}

// Validate the image of the tree edges (Alg. 4: 1-1 vertex map, delta range,
// edge order; the first failing check is the recorded cause), then count the
// motif instances that extend it (Alg. 5).
static int validate_and_derive(const or_prep& R, const int32_t* img_e /* indexed by motif edge */,
                               uint32_t* status, uint32_t* n_phi, u128* m_phi) {
    const or_graph& G = *R.g;
    const Plan& P = R.P;
    const or_motif& M = P.mo;
    *status = 0; *n_phi = 0; *m_phi = 0;
    int32_t img_v[8];
    for (int x = 0; x < M.k; ++x) img_v[x] = -1;
    for (int p : P.tree_sorted) {
        img_v[M.src[p]] = G.e[img_e[p]].u;
        img_v[M.dst[p]] = G.e[img_e[p]].v;
    }
    for (int x = 0; x < M.k; ++x)
        for (int y = x + 1; y < M.k; ++y)
            if (img_v[x] == img_v[y]) { *status = 1; return OR_OK; }
    int64_t tmin = 0, tmax = 0;
    bool firstt = true;
    for (int p : P.tree_sorted) {
        int64_t t = G.e[img_e[p]].t;
        if (firstt || t < tmin) tmin = t;
        if (firstt || t > tmax) tmax = t;
        firstt = false;
    }
    if (tmax - tmin > R.delta) { *status = 2; return OR_OK; }
    // every ordered pair of tree edges strictly in order
    for (int p : P.tree_sorted)
        for (int q : P.tree_sorted)
            if (precedes(P.R, p, q) && !(G.e[img_e[p]].t < G.e[img_e[q]].t)) {
                *status = 3;
                return OR_OK;
            }
    // N_phi: the number of intervals that contain every tree edge.  Only the
    // intervals starting at or before t_min and after t_min - 2*delta can.
    uint32_t cnt = 0;
    for (int64_t i = std::max<int64_t>(0, tmin / R.ilen - 1); i <= tmin / R.ilen + 1 && i < R.q; ++i)
        if (i * R.ilen <= tmin && tmax < (i + 2) * R.ilen) ++cnt;
    *n_phi = cnt;
    // Alg. 5: for each non-tree motif edge, the edges of G that can match it
    // (binary search on the multi-edge list to the times any completion can
    // use); tree edges are fixed single-element lists.  Lists are numbered in
    // pi order; ListCount counts strictly increasing chains.  The delta window
    // is enforced by fixing the first edge of the chain.
    std::vector<std::vector<int32_t>> lists(M.l);
    for (int p = 0; p < M.l; ++p) {
        if (P.in_tree[p]) { lists[p].push_back(img_e[p]); continue; }
        auto it = G.el.find({img_v[M.src[p]], img_v[M.dst[p]]});
        if (it == G.el.end()) return OR_OK;  // no edge can match p: M_phi = 0
        const std::vector<int32_t>& L = it->second;
        for (size_t x = first_at_or_after(G, L, tmax - R.delta); x < L.size(); ++x) {
            if (G.e[L[x]].t > tmin + R.delta) break;
            lists[p].push_back(L[x]);
        }
    }
    if (M.partial) {
        // A partial order: the completions are counted by their definition
        // (Def. "temporal match" with the order restricted to the given
        // pairs): every choice of one edge per list, each pair of the
        // relation strictly in order, distinct edges, all within delta.
        std::vector<int32_t> pick(M.l, -1);
        u128 total = 0;
        if (!po_enumerate(G, M, P.R, lists, 0, pick, &total)) return OR_EOVERFLOW;
        *m_phi = total;
        return OR_OK;
    }
    u128 total = 0;
    for (int32_t f : lists[0]) {
        u128 c;
        if (!list_count(G, lists, 1, G.e[f].t, G.e[f].t + R.delta, &c)) return OR_EOVERFLOW;
        if (!add_ok(total, c, &total)) return OR_EOVERFLOW;
    }
    *m_phi = total;
    return OR_OK;
}

extern "C" int or_derive_cnt(const or_prep* p, const int32_t* eids, or_u128* m_phi) {
    const Plan& P = p->P;
    int32_t img_e[16];
    for (int x = 0; x < 16; ++x) img_e[x] = -1;
    int32_t img_v[8];
    for (int x = 0; x < 8; ++x) img_v[x] = -1;
    for (size_t a = 0; a < P.tree_sorted.size(); ++a) {
        if (eids[a] < 0 || eids[a] >= p->g->m) return OR_EINVAL;
        int q = P.tree_sorted[a];
        img_e[q] = eids[a];
        // the tree edges must agree on the image of every shared vertex
        const int32_t ends[2] = {p->g->e[eids[a]].u, p->g->e[eids[a]].v};
        const int vs[2] = {P.mo.src[q], P.mo.dst[q]};
        for (int b = 0; b < 2; ++b) {
            if (img_v[vs[b]] >= 0 && img_v[vs[b]] != ends[b]) return OR_EINVAL;
            img_v[vs[b]] = ends[b];
        }
    }
    uint32_t st, np;
    u128 mp;
    int rc = validate_and_derive(*p, img_e, &st, &np, &mp);
    if (rc != OR_OK) return rc;
    if (st != 0) return OR_EINVAL;
    *m_phi = to_or(mp);
    return OR_OK;
}

// ------------------------------------------------------------------------
// Random instance listing (Sec. 4.3): the r-th completion of a valid tree
// image, completions ordered lexicographically by the eids of the motif's
// edges in pi order (tree edges fixed).
// ------------------------------------------------------------------------
static bool nth_completion(const or_graph& G, const std::vector<std::vector<int32_t>>& lists, size_t p,
                           int64_t after, int64_t t_first, int64_t delta, u128& r, std::vector<int32_t>& pick) {
    if (p == lists.size()) {
        if (r == 0) return true;
        --r;
        return false;
    }
    for (int32_t x : lists[p]) {
        const int64_t tx = G.e[x].t;
        if (tx <= after) continue;
        const int64_t tf = p == 0 ? tx : t_first;
        if (tx - tf > delta) continue;
        pick[p] = x;
        if (nth_completion(G, lists, p + 1, tx, tf, delta, r, pick)) return true;
    }
    return false;
}

extern "C" int or_list_instance(const or_prep* p, const int32_t* eids, or_u128 rank, int32_t* out) {
    if (!p || !eids || !out || p->P.mo.partial) return OR_EINVAL;
    const or_graph& G = *p->g;
    const Plan& P = p->P;
    const or_motif& M = P.mo;
    int32_t img_e[16];
    for (int x = 0; x < 16; ++x) img_e[x] = -1;
    int32_t img_v[8];
    for (int x = 0; x < 8; ++x) img_v[x] = -1;
    for (size_t a = 0; a < P.tree_sorted.size(); ++a) {
        if (eids[a] < 0 || eids[a] >= G.m) return OR_EINVAL;
        const int q = P.tree_sorted[a];
        img_e[q] = eids[a];
        img_v[M.src[q]] = G.e[eids[a]].u;
        img_v[M.dst[q]] = G.e[eids[a]].v;
    }
    uint32_t st, np;
    u128 mp;
    const int rc = validate_and_derive(*p, img_e, &st, &np, &mp);
    if (rc != OR_OK) return rc;
    u128 r = ((u128)rank.hi << 64) | rank.lo;
    if (st != 0 || r >= mp) return OR_EINVAL;
    int64_t tmin = 0, tmax = 0;
    bool firstt = true;
    for (int q : P.tree_sorted) {
        const int64_t t = G.e[img_e[q]].t;
        if (firstt || t < tmin) tmin = t;
        if (firstt || t > tmax) tmax = t;
        firstt = false;
    }
    // the candidate lists of Alg. 5: the tree edge itself, or the multi-edge
    // list of the non-tree edge's images within delta of the tree times
    std::vector<std::vector<int32_t>> lists(M.l);
    for (int q = 0; q < M.l; ++q) {
        if (P.in_tree[q]) {
            lists[q].push_back(img_e[q]);
            continue;
        }
        auto it = G.el.find({img_v[M.src[q]], img_v[M.dst[q]]});
        if (it == G.el.end()) return OR_EINVAL;
        for (size_t x = first_at_or_after(G, it->second, tmax - p->delta); x < it->second.size(); ++x) {
            if (G.e[it->second[x]].t > tmin + p->delta) break;
            lists[q].push_back(it->second[x]);
        }
    }
    std::vector<int32_t> pick(M.l, -1);
    if (!nth_completion(G, lists, 0, INT64_MIN, 0, p->delta, r, pick)) return OR_EINVAL;
    for (int q = 0; q < M.l; ++q) out[q] = pick[q];
    return OR_OK;
}

// ------------------------------------------------------------------------
// Alg. 3 (SampleSubg) and Alg. 6 (Estimate).
// ------------------------------------------------------------------------

// Inverse CDF: the unique index x with sum(w[0..x)) <= r < sum(w[0..x]).
static size_t pick(const std::vector<u128>& wts, u128 r) {
    u128 cum = 0;
    for (size_t x = 0; x < wts.size(); ++x) {
        if (r < cum + wts[x]) return x;
        cum += wts[x];
    }
    return wts.size();  // unreachable when r < total
}

// ------------------------------------------------------------------------
// Standard error of the estimate (Sec. 4.4, Lemma "unbiased-estimate": the
// estimate is (W / 2) times the mean of the per-sample terms Y = 2 M_phi /
// N_phi, so its standard error is (W / 2) s / sqrt(k) with s^2 the unbiased
// sample variance of Y).  s^2 = D / (k (k - 1)) with D = k sum Y^2 - (sum Y)^2,
// an exact non-negative integer below 2^256, formed here with 32-bit limbs
// and rounded once to the nearest double (ties to even).
// ------------------------------------------------------------------------
namespace {
struct Big {  // little-endian 32-bit limbs, 256 bits
    uint32_t d[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};

Big big_of(u128 x) {
    Big b;
    for (int i = 0; i < 4; ++i) b.d[i] = (uint32_t)(x >> (32 * i));
    return b;
}

// schoolbook product; both factors below 2^128, so it fits 256 bits
Big big_mul(const Big& a, const Big& b) {
    uint64_t acc[16] = {0};
    for (int i = 0; i < 8; ++i)
        for (int j = 0; i + j < 8; ++j) {
            uint64_t p = (uint64_t)a.d[i] * b.d[j];
            // add p at limb i + j, carrying upward
            int at = i + j;
            while (p != 0 && at < 8) {
                uint64_t s = acc[at] + (p & 0xffffffffu);
                acc[at] = s & 0xffffffffu;
                p = (p >> 32) + (s >> 32);
                ++at;
            }
        }
    Big r;
    for (int i = 0; i < 8; ++i) r.d[i] = (uint32_t)acc[i];
    return r;
}

// a - b, requires a >= b; returns false (and 0) otherwise
bool big_sub(const Big& a, const Big& b, Big* r) {
    int64_t borrow = 0;
    for (int i = 0; i < 8; ++i) {
        int64_t x = (int64_t)a.d[i] - (int64_t)b.d[i] - borrow;
        borrow = x < 0 ? 1 : 0;
        r->d[i] = (uint32_t)(x + (borrow << 32));
    }
    if (borrow) {
        *r = Big();
        return false;
    }
    return true;
}

bool big_bit(const Big& a, int i) { return (a.d[i / 32] >> (i % 32)) & 1u; }

// nearest double, ties to even: the 53 bits below and at the top set bit,
// then the next bit (half) and whether any bit below it is set (sticky)
double big_to_double(const Big& a) {
    int top = -1;
    for (int i = 255; i >= 0 && top < 0; --i)
        if (big_bit(a, i)) top = i;
    if (top < 0) return 0.0;
    uint64_t mant = 0;
    const int low = top - 52;  // bit position of the mantissa's last bit
    for (int i = top; i >= (low > 0 ? low : 0); --i) mant = (mant << 1) | (big_bit(a, i) ? 1u : 0u);
    if (low <= 0) return std::ldexp((double)mant, low < 0 ? 0 : low);
    const bool half = big_bit(a, low - 1);
    bool sticky = false;
    for (int i = low - 2; i >= 0; --i) sticky = sticky || big_bit(a, i);
    if (half && (sticky || (mant & 1u))) ++mant;  // may carry to 2^53: still exact
    return std::ldexp((double)mant, low);
}
}  // namespace

static double std_error_of(u128 W, u128 acc2, u128 acc2_sq, uint64_t k, uint32_t flags) {
    if (k < 2 || W == 0 || (flags & 2u)) return 0.0;
    Big D;
    if (!big_sub(big_mul(big_of((u128)k), big_of(acc2_sq)), big_mul(big_of(acc2), big_of(acc2)), &D))
        return 0.0;  // D < 0 cannot happen for sums over at most k samples
    const double Dd = big_to_double(D);
    const double kd = (double)k;
    const double km1 = (double)(k - 1);
    const double var = Dd / (kd * km1);
    return ((double)W / 2.0) * std::sqrt(var / kd);
}

extern "C" double or_std_error(or_u128 W, or_u128 acc2, or_u128 acc2_sq, uint64_t k, uint32_t flags) {
    return std_error_of(from_or(W), from_or(acc2), from_or(acc2_sq), k, flags);
}

extern "C" int or_sample(const or_prep* p, uint64_t seed, uint64_t j0, uint64_t count,
                         uint64_t k_total, or_result* res, or_rec* recs) {
    if (!p || !res) return OR_EINVAL;
    const or_prep& R = *p;
    const Plan& P = R.P;
    std::memset(res, 0, sizeof *res);
    res->W = to_or(R.W);
    res->k = k_total;
    res->q = R.q;
    if (R.W == 0) {
        res->flags |= 1u;
        res->estimate = 0.0;
        for (uint64_t a = 0; recs && a < count; ++a) {
            std::memset(&recs[a], 0, sizeof(or_rec));
            recs[a].status = 4;  // not drawn: there is nothing to sample
            for (int x = 0; x < 8; ++x) recs[a].eid[x] = -1;
        }
        return OR_OK;
    }
    u128 acc2 = 0, acc2_sq = 0;
    std::vector<int32_t> cand;
    std::vector<u128> wts;
    for (uint64_t a = 0; a < count; ++a) {
        uint64_t j = j0 + a;
        int32_t img_e[16];
        for (int x = 0; x < 16; ++x) img_e[x] = -1;
        // Alg. 6: pick G_i with probability W_i / W; Alg. 3: pick the center
        // edge with probability w_{c,e} / W_i -- one draw, split in two stages.
        u128 r0 = draw(seed, j, 0, R.W);
        int64_t i = (int64_t)(std::upper_bound(R.cumW.begin(), R.cumW.end(), r0) - R.cumW.begin()) - 1;
        u128 r = r0 - R.cumW[i];
        const std::vector<u128>& rc = R.root_cum[i];
        int64_t x = (int64_t)(std::upper_bound(rc.begin(), rc.end(), r) - rc.begin()) - 1;
        img_e[P.center] = (int32_t)(R.lo[i] + x);
        // Alg. 3: top-down, each child with probability proportional to its
        // weight over its candidate list.
        uint32_t d = 1;
        for (size_t step = 1; step < P.preorder.size(); ++step) {
            int c = P.preorder[step];
            int s = P.parent[c];
            candidates(R, i, s, img_e[s], c, cand);
            wts.clear();
            u128 Wx = 0;
            for (int32_t f : cand) {
                wts.push_back(weight(R, i, c, f));
                Wx += wts.back();
            }
            // A child of an edge with positive weight always has positive
            // candidate weight (the parent's weight is their product).
            if (Wx == 0) return OR_EINVAL;
            u128 rr = draw(seed, j, d++, Wx);
            img_e[c] = cand[pick(wts, rr)];
        }
        uint32_t status, n_phi;
        u128 m_phi;
        int rcode = validate_and_derive(R, img_e, &status, &n_phi, &m_phi);
        if (rcode != OR_OK) return rcode;
        if (status == 0) {
            ++res->n_valid;
            if (m_phi != 0) ++res->n_nonzero;
            // 2 * M_phi / N_phi with N_phi in {1, 2} stays an integer.
            u128 term;
            if (!mul_ok(m_phi, (u128)(2 / n_phi), &term)) return OR_EOVERFLOW;
            if (!add_ok(acc2, term, &acc2)) return OR_EOVERFLOW;
            u128 sq;
            if (!mul_ok(term, term, &sq) || !add_ok(acc2_sq, sq, &acc2_sq)) {
                acc2_sq = ~(u128)0;
                res->flags |= 2u;
            }
        } else if (status == 1) {
            ++res->n_bad_vertex;
        } else if (status == 2) {
            ++res->n_bad_delta;
        } else {
            ++res->n_bad_order;
        }
        if (recs) {
            or_rec& out = recs[a];
            std::memset(&out, 0, sizeof out);
            out.interval = (uint32_t)i;
            out.status = status;
            out.n_phi = status == 0 ? n_phi : 0;
            for (int y = 0; y < 8; ++y) out.eid[y] = -1;
            for (size_t y = 0; y < P.tree_sorted.size(); ++y) out.eid[y] = img_e[P.tree_sorted[y]];
            out.m_phi = to_or(status == 0 ? m_phi : 0);
        }
    }
    res->acc2 = to_or(acc2);
    res->acc2_sq = to_or(acc2_sq);
    // Alg. 6: C^ = (cnt / k) * W with cnt = acc2 / 2.
    res->estimate = k_total ? (double)R.W * ((double)acc2 / (2.0 * (double)k_total)) : 0.0;
    res->std_error = std_error_of(R.W, acc2, acc2_sq, k_total, res->flags);
    return OR_OK;
}
