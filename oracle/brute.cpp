// TIMEST reference oracle -- TEST INFRASTRUCTURE ONLY (see timest_oracle.h).
//
// Brute-force enumerators written straight from the definitions.  They share
// the graph container with oracle.cpp but none of its algorithms: no weights,
// no candidate lists, no ListCount.  Every candidate edge is found by scanning,
// every condition is checked as the definition states it.

#include "timest_oracle.h"
#include "graph_internal.h"

#include <algorithm>
#include <cstring>
#include <map>
#include <utility>
#include <vector>

typedef unsigned __int128 u128;
static or_u128 to_or(u128 x) { return or_u128{(uint64_t)x, (uint64_t)(x >> 64)}; }

// ------------------------------------------------------------------------
// Exact count C (Def. "temporal match"): 1-1 vertex and edge maps, edges
// mapped with direction, times strictly increasing in pi order, every pair of
// times within delta.  Backtracking over the motif edges in pi order.
// ------------------------------------------------------------------------
// The time constraints of a motif as a relation: before_of(mo, p, q) is true
// when edge p must be strictly earlier than edge q -- every p < q for the
// total order of the list; for a partial order, the given pairs and every
// pair they imply through a chain of given pairs.
static bool before_of(const or_motif* mo, int p, int q) {
    if (p < 0 || q < 0 || p >= mo->l || q >= mo->l || p == q) return false;
    if (!mo->partial) return p < q;
    // reachability from p to q along given pairs (depth-first)
    bool seen[16] = {false};
    int stack[16], top = 0;
    stack[top++] = p;
    seen[p] = true;
    while (top > 0) {
        const int a = stack[--top];
        for (int b = 0; b < mo->l; ++b) {
            if (seen[b] || !((mo->before[b] >> a) & 1u)) continue;
            if (b == q) return true;
            seen[b] = true;
            stack[top++] = b;
        }
    }
    return false;
}

struct CountCtx {
    const or_graph* g;
    const or_motif* mo;
    int32_t img[8];
    int64_t t0;
    u128 count;
    int32_t eid[16];  // partial orders: the edge matched to each motif edge so far
};

// Partial orders: motif edges in list order, each over every edge of G; an
// edge is kept when the vertex map stays consistent and 1-1, it differs from
// the edges matched so far, every constraint with an earlier matched edge
// holds, and all matched times stay within delta.
static void count_po_rec(CountCtx& C, int p) {
    const or_motif& M = *C.mo;
    if (p == M.l) { ++C.count; return; }
    const int x = M.src[p], y = M.dst[p];
    for (int64_t id = 0; id < C.g->m; ++id) {
        const OEdge& E = C.g->e[id];
        bool ok = true;
        for (int z = 0; z < M.k && ok; ++z) {
            if (z == x || z == y || C.img[z] < 0) continue;
            if (C.img[z] == E.u || C.img[z] == E.v) ok = false;
        }
        if (!ok) continue;
        if (C.img[x] >= 0 && C.img[x] != E.u) continue;
        if (C.img[y] >= 0 && C.img[y] != E.v) continue;
        for (int q = 0; q < p && ok; ++q) {
            const OEdge& F = C.g->e[C.eid[q]];
            if (C.eid[q] == id) ok = false;
            if (before_of(&M, q, p) && !(F.t < E.t)) ok = false;
            if (before_of(&M, p, q) && !(E.t < F.t)) ok = false;
            if (F.t - E.t > M.delta || E.t - F.t > M.delta) ok = false;
        }
        if (!ok) continue;
        const int32_t sx = C.img[x], sy = C.img[y];
        C.img[x] = E.u;
        C.img[y] = E.v;
        C.eid[p] = (int32_t)id;
        count_po_rec(C, p + 1);
        C.eid[p] = -1;
        C.img[x] = sx;
        C.img[y] = sy;
    }
}

static void count_rec(CountCtx& C, int p, int64_t tprev) {
    const or_motif& M = *C.mo;
    if (p == M.l) { ++C.count; return; }
    int x = M.src[p], y = M.dst[p];
    // eids are in time order: scan every edge strictly after the previous
    // matched edge and no later than t0 + delta
    int64_t start = 0;
    if (p > 0) {
        int64_t a = 0, b = C.g->m;
        while (a < b) { int64_t mid = (a + b) / 2; if (C.g->e[mid].t <= tprev) a = mid + 1; else b = mid; }
        start = a;
    }
    for (int64_t id = start; id < C.g->m; ++id) {
        const OEdge& E = C.g->e[id];
        if (p > 0 && E.t - C.t0 > C.mo->delta) break;
        // map x -> E.u and y -> E.v consistently and injectively
        bool ok = true;
        for (int z = 0; z < M.k && ok; ++z) {
            if (z == x || z == y || C.img[z] < 0) continue;
            if (C.img[z] == E.u || C.img[z] == E.v) ok = false;
        }
        if (!ok) continue;
        if (C.img[x] >= 0 && C.img[x] != E.u) continue;
        if (C.img[y] >= 0 && C.img[y] != E.v) continue;
        int32_t sx = C.img[x], sy = C.img[y];
        C.img[x] = E.u;
        C.img[y] = E.v;
        int64_t st0 = C.t0;
        if (p == 0) C.t0 = E.t;
        count_rec(C, p + 1, E.t);
        C.t0 = st0;
        C.img[x] = sx;
        C.img[y] = sy;
    }
}

static bool motif_basic_ok(const or_motif* mo) {
    if (!mo || mo->k < 2 || mo->k > 8 || mo->l < 1 || mo->l > 16 || mo->delta < 1) return false;
    for (int p = 0; p < mo->l; ++p)
        if (mo->src[p] < 0 || mo->src[p] >= mo->k || mo->dst[p] < 0 || mo->dst[p] >= mo->k ||
            mo->src[p] == mo->dst[p])
            return false;
    if (mo->partial > 1) return false;
    if (mo->partial) {
        for (int q = 0; q < 16; ++q)
            for (int p = 0; p < 16; ++p)
                if (((mo->before[q] >> p) & 1u) && (p >= q || q >= mo->l)) return false;
        for (int p = 0; p < mo->l; ++p)
            for (int q = p + 1; q < mo->l; ++q)
                if (mo->src[p] == mo->src[q] && mo->dst[p] == mo->dst[q] && !before_of(mo, p, q)) return false;
    }
    return true;
}

extern "C" int or_brute_count(const or_graph* g, const or_motif* mo, or_u128* out) {
    if (!g || !out || !motif_basic_ok(mo)) return OR_EINVAL;
    CountCtx C;
    C.g = g;
    C.mo = mo;
    for (int z = 0; z < 8; ++z) C.img[z] = -1;
    C.t0 = 0;
    C.count = 0;
    for (int z = 0; z < 16; ++z) C.eid[z] = -1;
    if (mo->partial)
        count_po_rec(C, 0);
    else
        count_rec(C, 0, 0);
    *out = to_or(C.count);
    return OR_OK;
}

// ------------------------------------------------------------------------
// delta-partial matches of a spanning tree (the unlabelled definition in
// Sec. 4 after Def. "spanning tree"): a homomorphism of the tree into G in
// which every parent/child pair of tree edges (a) shares exactly one vertex of
// G and (b) has the child's time in [t, t+delta] when the child follows the
// parent in pi, in [t-delta, t] otherwise.
// ------------------------------------------------------------------------
struct Tree {
    int l;
    const or_motif* mo;
    bool in_tree[16];
    int parent[16];
    int order[8];       // tree edges, every parent before its children
    int n_order;
    int sorted[8];      // tree edges by pi index
    int n_sorted;
};

static bool build_tree(const or_motif* mo, const or_tree* tr, Tree& T) {
    T.l = mo->l;
    T.mo = mo;
    for (int p = 0; p < 16; ++p) { T.in_tree[p] = false; T.parent[p] = -2; }
    if (!tr || tr->n_edges != mo->k - 1) return false;
    for (int j = 0; j < tr->n_edges; ++j) {
        if (tr->edge[j] < 0 || tr->edge[j] >= mo->l) return false;
        T.in_tree[tr->edge[j]] = true;
    }
    if (!T.in_tree[tr->center]) return false;
    // breadth-first from the center edge over shared vertices
    T.parent[tr->center] = -1;
    T.order[0] = tr->center;
    T.n_order = 1;
    for (int head = 0; head < T.n_order; ++head) {
        int s = T.order[head];
        for (int p = 0; p < mo->l; ++p) {
            if (!T.in_tree[p] || T.parent[p] != -2) continue;
            bool touches = mo->src[p] == mo->src[s] || mo->src[p] == mo->dst[s] ||
                           mo->dst[p] == mo->src[s] || mo->dst[p] == mo->dst[s];
            if (!touches) continue;
            // the vertex shared with s must not be the one s shares with its parent
            if (T.parent[s] >= 0) {
                int q = T.parent[s];
                int z = -1;  // vertex of s shared with its parent
                if (mo->src[s] == mo->src[q] || mo->src[s] == mo->dst[q]) z = mo->src[s];
                else z = mo->dst[s];
                int lowv = (z == mo->src[s]) ? mo->dst[s] : mo->src[s];
                if (mo->src[p] != lowv && mo->dst[p] != lowv) continue;
            }
            T.parent[p] = s;
            if (T.n_order >= 8) return false;
            T.order[T.n_order++] = p;
        }
    }
    if (T.n_order != tr->n_edges) return false;
    T.n_sorted = 0;
    for (int p = 0; p < mo->l; ++p)
        if (T.in_tree[p]) T.sorted[T.n_sorted++] = p;
    return true;
}

static int shared_vertices(const OEdge& a, const OEdge& b) {
    int c = 0;
    if (a.u == b.u || a.u == b.v) ++c;
    if (a.v == b.u || a.v == b.v) ++c;
    return c;
}

struct PMCtx {
    const or_graph* g;
    const Tree* T;
    int64_t delta;
    int64_t ilo, ihi;          // allowed time range [ilo, ihi) for every tree edge
    int32_t img_v[8];
    int32_t img_e[16];
    int first;                 // index in T->order where the enumeration starts
    bool exclude;              // constraint 2: a child shares exactly one vertex with its parent
    // collection of whole matches (optional)
    std::vector<std::vector<int32_t>>* found;
    u128 count;
};

static bool parent_child_ok(const PMCtx& C, int s, int c, const OEdge& Ep, const OEdge& Ec) {
    const int sh = shared_vertices(Ep, Ec);
    if (C.exclude ? sh != 1 : sh < 1) return false;
    const or_motif* mo = C.T->mo;
    if (before_of(mo, s, c)) return Ec.t >= Ep.t && Ec.t <= Ep.t + C.delta;
    if (before_of(mo, c, s)) return Ec.t >= Ep.t - C.delta && Ec.t <= Ep.t;
    return Ec.t >= Ep.t - C.delta && Ec.t <= Ep.t + C.delta;  // unordered pair
}

static void pm_rec(PMCtx& C, int idx) {
    const Tree& T = *C.T;
    const or_motif& M = *T.mo;
    if (idx == T.n_order) {
        ++C.count;
        if (C.found) {
            std::vector<int32_t> v(T.n_sorted);
            for (int a = 0; a < T.n_sorted; ++a) v[a] = C.img_e[T.sorted[a]];
            C.found->push_back(v);
        }
        return;
    }
    int p = T.order[idx];
    int s = T.parent[p];
    // only edges below the subtree root are enumerated here
    bool in_sub = false;
    for (int q = p; q >= 0; q = T.parent[q])
        if (q == T.order[C.first]) in_sub = true;
    if (!in_sub) { pm_rec(C, idx + 1); return; }
    for (int64_t id = 0; id < C.g->m; ++id) {
        const OEdge& E = C.g->e[id];
        if (E.t < C.ilo || E.t >= C.ihi) continue;
        int x = M.src[p], y = M.dst[p];
        if (C.img_v[x] >= 0 && C.img_v[x] != E.u) continue;
        if (C.img_v[y] >= 0 && C.img_v[y] != E.v) continue;
        if (idx > C.first && !parent_child_ok(C, s, p, C.g->e[C.img_e[s]], E)) continue;
        int32_t sx = C.img_v[x], sy = C.img_v[y];
        C.img_v[x] = E.u;
        C.img_v[y] = E.v;
        C.img_e[p] = (int32_t)id;
        pm_rec(C, idx + 1);
        C.img_e[p] = -1;
        C.img_v[x] = sx;
        C.img_v[y] = sy;
    }
}

static void pm_init(PMCtx& C, const or_graph* g, const Tree* T, int64_t delta, int64_t ilo, int64_t ihi) {
    C.g = g;
    C.T = T;
    C.delta = delta;
    C.ilo = ilo;
    C.ihi = ihi;
    for (int z = 0; z < 8; ++z) C.img_v[z] = -1;
    for (int z = 0; z < 16; ++z) C.img_e[z] = -1;
    C.first = 0;
    C.exclude = true;
    C.found = nullptr;
    C.count = 0;
}

// Interval unit under the constraint flags: delta with constraint 3, else one
// interval over the whole span.
static int64_t unit_of(const or_graph* g, const or_motif* mo, uint32_t flags) {
    return (flags & OR_C_WINDOWS) ? mo->delta : g->T + 1;
}

extern "C" int or_brute_tree_weight(const or_graph* g, const or_motif* mo, const or_tree* tr, or_u128* W) {
    return or_brute_tree_weight_ex(g, mo, tr, OR_C_ALL, W);
}

extern "C" int or_brute_tree_weight_ex(const or_graph* g, const or_motif* mo, const or_tree* tr, uint32_t flags,
                                       or_u128* W) {
    if (!g || !W || !motif_basic_ok(mo)) return OR_EINVAL;
    Tree T;
    if (!build_tree(mo, tr, T)) return OR_EINVAL;
    u128 total = 0;
    const int64_t L = unit_of(g, mo, flags);
    int64_t q = g->m > 0 ? g->T / L + 1 : 0;
    for (int64_t i = 0; i < q; ++i) {
        PMCtx C;
        pm_init(C, g, &T, mo->delta, i * L, (i + 2) * L);
        C.exclude = (flags & OR_C_EXCLUDE) != 0;
        pm_rec(C, 0);
        total += C.count;
    }
    *W = to_or(total);
    return OR_OK;
}

extern "C" int or_brute_edge_weight(const or_graph* g, const or_motif* mo, const or_tree* tr,
                                    int64_t interval, int32_t s, int32_t eid, or_u128* w) {
    if (!g || !w || !motif_basic_ok(mo) || eid < 0 || eid >= g->m) return OR_EINVAL;
    Tree T;
    if (!build_tree(mo, tr, T)) return OR_EINVAL;
    int pos = -1;
    for (int a = 0; a < T.n_order; ++a)
        if (T.order[a] == s) pos = a;
    if (pos < 0) return OR_EINVAL;
    PMCtx C;
    pm_init(C, g, &T, mo->delta, interval * mo->delta, (interval + 2) * mo->delta);
    const OEdge& E = g->e[eid];
    if (E.t < C.ilo || E.t >= C.ihi) return OR_EINVAL;
    C.first = pos;
    C.img_v[mo->src[s]] = E.u;
    C.img_v[mo->dst[s]] = E.v;
    C.img_e[s] = eid;
    pm_rec(C, pos + 1);
    *w = to_or(C.count);
    return OR_OK;
}

// Completions of a tree image: every assignment of the non-tree motif edges
// to edges of G such that the whole map is an M-match (Def. "temporal match").
static void completion_rec(const or_graph* g, const or_motif* mo, const Tree& T, int32_t* img_e,
                           const int32_t* img_v, int p, u128* count) {
    if (p == mo->l) {
        // every constrained pair strictly in order, distinct edges (the edge
        // map is 1-1), every pair of times within delta
        for (int a = 0; a < mo->l; ++a)
            for (int b = 0; b < mo->l; ++b) {
                if (a == b) continue;
                if (img_e[a] == img_e[b]) return;
                const int64_t ta = g->e[img_e[a]].t, tb = g->e[img_e[b]].t;
                if (before_of(mo, a, b) && !(ta < tb)) return;
                if (tb - ta > mo->delta) return;
            }
        ++*count;
        return;
    }
    if (T.in_tree[p]) { completion_rec(g, mo, T, img_e, img_v, p + 1, count); return; }
    for (int64_t id = 0; id < g->m; ++id) {
        const OEdge& E = g->e[id];
        if (E.u != img_v[mo->src[p]] || E.v != img_v[mo->dst[p]]) continue;
        img_e[p] = (int32_t)id;
        completion_rec(g, mo, T, img_e, img_v, p + 1, count);
        img_e[p] = -1;
    }
}

extern "C" int64_t or_brute_partial_matches(const or_graph* g, const or_motif* mo, const or_tree* tr,
                                            int64_t cap, int32_t* eids, uint32_t* n_phi,
                                            uint32_t* status, or_u128* m_phi_brute) {
    return or_brute_partial_matches_ex(g, mo, tr, OR_C_ALL, cap, eids, n_phi, status, m_phi_brute);
}

extern "C" int64_t or_brute_partial_matches_ex(const or_graph* g, const or_motif* mo, const or_tree* tr,
                                               uint32_t flags, int64_t cap, int32_t* eids, uint32_t* n_phi,
                                               uint32_t* status, or_u128* m_phi_brute) {
    if (!g || !motif_basic_ok(mo)) return OR_EINVAL;
    Tree T;
    if (!build_tree(mo, tr, T)) return OR_EINVAL;
    std::vector<std::vector<int32_t>> found;
    PMCtx C;
    pm_init(C, g, &T, mo->delta, INT64_MIN, INT64_MAX);
    C.exclude = (flags & OR_C_EXCLUDE) != 0;
    C.found = &found;
    pm_rec(C, 0);
    const int64_t L = unit_of(g, mo, flags);
    int64_t q = g->m > 0 ? g->T / L + 1 : 0;
    for (int64_t a = 0; a < (int64_t)found.size() && a < cap; ++a) {
        const std::vector<int32_t>& f = found[a];
        int32_t img_e[16];
        int32_t img_v[8];
        for (int z = 0; z < 16; ++z) img_e[z] = -1;
        for (int z = 0; z < 8; ++z) img_v[z] = -1;
        int64_t tmin = INT64_MAX, tmax = INT64_MIN;
        for (int b = 0; b < T.n_sorted; ++b) {
            int p = T.sorted[b];
            const OEdge& E = g->e[f[b]];
            img_e[p] = f[b];
            img_v[mo->src[p]] = E.u;
            img_v[mo->dst[p]] = E.v;
            tmin = std::min(tmin, E.t);
            tmax = std::max(tmax, E.t);
            if (eids) eids[a * 8 + b] = f[b];
        }
        for (int b = T.n_sorted; b < 8 && eids; ++b) eids[a * 8 + b] = -1;
        // intervals I_i that hold every tree edge
        uint32_t np = 0;
        for (int64_t i = 0; i < q; ++i)
            if (tmin >= i * L && tmax < (i + 2) * L) ++np;
        if (n_phi) n_phi[a] = np;
        // literal validation, first failing cause
        uint32_t st = 0;
        for (int x = 0; x < mo->k && st == 0; ++x)
            for (int y = x + 1; y < mo->k; ++y)
                if (img_v[x] == img_v[y]) { st = 1; break; }
        if (st == 0 && tmax - tmin > mo->delta) st = 2;
        for (int a2 = 0; a2 < T.n_sorted && st == 0; ++a2)
            for (int b = 0; b < T.n_sorted; ++b)
                if (before_of(mo, T.sorted[a2], T.sorted[b]) && !(g->e[f[a2]].t < g->e[f[b]].t)) { st = 3; break; }
        if (status) status[a] = st;
        u128 cnt = 0;
        bool injective = true;
        for (int x = 0; x < mo->k; ++x)
            for (int y = x + 1; y < mo->k; ++y)
                if (img_v[x] == img_v[y]) injective = false;
        if (injective) completion_rec(g, mo, T, img_e, img_v, 0, &cnt);
        if (m_phi_brute) m_phi_brute[a] = to_or(cnt);
    }
    return (int64_t)found.size();
}
