// C ABI of the TIMEST GPU library: argument checks, the motif plan, handle
// lifetimes and the host side of each entry point.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "tm_internal.h"

static thread_local char g_last_error[512] = "";

int tm_fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
    return code;
}

static std::mutex g_prof_mu;
static bool g_prof_on = false;
static uint32_t g_prof_mask = (1u << TM_N_STAGES) - 1;
static tm_profile g_prof = {};

static thread_local bool t_prof_suspended = false;

void prof_suspend(bool on) { t_prof_suspended = on; }
bool prof_suspended() { return t_prof_suspended; }

bool prof_enabled(int stage) {
    if (t_prof_suspended || stage < 0 || stage >= TM_N_STAGES) return false;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    return g_prof_on && ((g_prof_mask >> stage) & 1u);
}

void prof_add(int stage, double ms) {
    if (stage < 0 || stage >= TM_N_STAGES) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.ms[stage] += ms;
    g_prof.launches[stage] += 1;
}

extern "C" int tm_release_cached(void) {
    dev_cache_trim();
    return TM_OK;
}

extern "C" void tm_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
}

extern "C" void tm_profile_stages(uint32_t mask) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_mask = mask & ((1u << TM_N_STAGES) - 1);
}

extern "C" int tm_profile_read(tm_profile* out, int reset) {
    if (!out) return tm_fail(TM_EINVAL, "profile_read: NULL");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    *out = g_prof;
    if (reset) g_prof = tm_profile{};
    return TM_OK;
}

int DevArena::alloc(void** p, size_t nbytes) {
    *p = nullptr;
    if (nbytes == 0) nbytes = 16;
    nbytes = (nbytes + 255) & ~(size_t)255;
    hipError_t e = dev_alloc(p, nbytes, stream);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return tm_fail(e == hipErrorOutOfMemory ? TM_ENOMEM : TM_EDEVICE,
                       "hipMalloc(%zu bytes): %s", nbytes, hipGetErrorString(e));
    }
    blocks.push_back(*p);
    bytes += nbytes;
    return TM_OK;
}

void DevArena::release_one(void* p, size_t nbytes) {
    for (size_t x = 0; x < blocks.size(); ++x) {
        if (blocks[x] != p) continue;
        blocks.erase(blocks.begin() + (long)x);
        bytes -= (nbytes ? (nbytes + 255) & ~(size_t)255 : 256);
        (void)dev_free(p, stream);
        return;
    }
}

// Called when no work of the library is in flight (every entry point
// synchronises before it returns), so the blocks are free for any stream.
void DevArena::release() {
    for (void* p : blocks) (void)dev_free(p, stream);
    if (!blocks.empty()) dev_stream_synced(stream);
    blocks.clear();
    bytes = 0;
}

// ---------------------------------------------------------------------------
// Motif and tree checks, and the rooted plan.
// ---------------------------------------------------------------------------
// The motif's "strictly earlier" relation: rel[q] holds p when edge p must
// precede edge q.  The total order: every p < q; a partial order: the given
// pairs closed under transitivity (pairs run from lower to higher index, so
// one pass in index order closes them).
static void order_closure(const tm_motif* mo, uint32_t rel[TM_MAX_L]) {
    for (int q = 0; q < TM_MAX_L; ++q) {
        if (q >= mo->l) {
            rel[q] = 0;
        } else if (!mo->partial) {
            rel[q] = (1u << q) - 1u;
        } else {
            uint32_t r = mo->before[q];
            for (int p = 0; p < q; ++p)
                if ((mo->before[q] >> p) & 1u) r |= rel[p];
            rel[q] = r;
        }
    }
}

// A partial order that orders every pair is the total order of the list.
static bool order_is_total(const tm_motif* mo, const uint32_t rel[TM_MAX_L]) {
    for (int q = 0; q < mo->l; ++q)
        if (rel[q] != (1u << q) - 1u) return false;
    return true;
}

int motif_check(const tm_motif* mo) {
    if (!mo) return tm_fail(TM_EINVAL, "motif: NULL");
    if (mo->partial > 1) return tm_fail(TM_EINVAL, "motif: partial = %u (0 or 1)", mo->partial);
    if (mo->k < 2 || mo->k > TM_MAX_K) return tm_fail(TM_EINVAL, "motif: k = %d outside [2, 8]", mo->k);
    if (mo->l < 1 || mo->l > TM_MAX_L) return tm_fail(TM_EINVAL, "motif: l = %d outside [1, 16]", mo->l);
    if (mo->delta < 1 || mo->delta >= ((int64_t)1 << 62))
        return tm_fail(TM_EINVAL, "motif: delta = %lld outside [1, 2^62)", (long long)mo->delta);
    int root[TM_MAX_K];
    for (int x = 0; x < mo->k; ++x) root[x] = x;
    auto find = [&](int x) {
        while (root[x] != x) x = root[x];
        return x;
    };
    for (int p = 0; p < mo->l; ++p) {
        const int a = mo->src[p], b = mo->dst[p];
        if (a < 0 || a >= mo->k || b < 0 || b >= mo->k)
            return tm_fail(TM_EINVAL, "motif: edge %d has an endpoint outside [0, k)", p);
        if (a == b) return tm_fail(TM_EINVAL, "motif: edge %d is a self loop", p);
        root[find(a)] = find(b);
    }
    for (int x = 1; x < mo->k; ++x)
        if (find(x) != find(0)) return tm_fail(TM_EINVAL, "motif: not weakly connected");
    if (mo->partial) {
        for (int q = 0; q < TM_MAX_L; ++q) {
            const uint32_t allowed = q < mo->l ? (1u << q) - 1u : 0u;
            if (mo->before[q] & ~allowed)
                return tm_fail(TM_EINVAL, "motif: before[%d] names an edge that is not listed earlier", q);
        }
        uint32_t rel[TM_MAX_L];
        order_closure(mo, rel);
        for (int p = 0; p < mo->l; ++p)
            for (int q = p + 1; q < mo->l; ++q)
                if (mo->src[p] == mo->src[q] && mo->dst[p] == mo->dst[q] && !((rel[q] >> p) & 1u))
                    return tm_fail(TM_EINVAL, "motif: parallel edges %d and %d are unordered", p, q);
        if (!order_is_total(mo, rel) && mo->l - (mo->k - 1) > kPoMaxFree)
            return tm_fail(TM_EINVAL, "motif: a partial order with more than %d non-tree edges", kPoMaxFree);
    }
    return TM_OK;
}

static bool spanning_tree_of(const tm_motif* mo, const int32_t* e, int cnt) {
    if (cnt != mo->k - 1) return false;
    int root[TM_MAX_K];
    for (int x = 0; x < mo->k; ++x) root[x] = x;
    auto find = [&](int x) {
        while (root[x] != x) x = root[x];
        return x;
    };
    for (int j = 0; j < cnt; ++j) {
        if (e[j] < 0 || e[j] >= mo->l) return false;
        const int a = find(mo->src[e[j]]), b = find(mo->dst[e[j]]);
        if (a == b) return false;  // repeated edge or cycle
        root[a] = b;
    }
    return true;
}

int plan_build(const tm_motif* mo, const tm_tree* tr, HostPlan* P) {
    TM_TRY(motif_check(mo));
    if (!tr) return tm_fail(TM_EINVAL, "tree: NULL");
    if (!spanning_tree_of(mo, tr->edge, tr->n_edges))
        return tm_fail(TM_EINVAL, "tree: not a spanning tree of the motif");
    bool in_tree[TM_MAX_L] = {false};
    for (int j = 0; j < tr->n_edges; ++j) in_tree[tr->edge[j]] = true;
    if (tr->center < 0 || tr->center >= mo->l || !in_tree[tr->center])
        return tm_fail(TM_EINVAL, "tree: center %d is not a tree edge", tr->center);
    HostPlan& H = *P;
    H = HostPlan();
    H.mo = *mo;
    H.tree = *tr;
    uint32_t rel[TM_MAX_L];
    order_closure(mo, rel);
    H.po = mo->partial && !order_is_total(mo, rel);
    if (!H.po) {  // the total order of the list, however it was given
        H.mo.partial = 0;
        std::memset(H.mo.before, 0, sizeof H.mo.before);
    }
    auto earlier = [&](int p, int q) { return ((rel[q] >> p) & 1u) != 0; };
    H.nt = tr->n_edges;
    for (int p = 0; p < TM_MAX_L; ++p) H.slot_of_edge[p] = -1;
    for (int s = 0; s < kMaxSlots; ++s) {
        H.n_children[s] = 0;
        H.height[s] = 0;
    }
    // Pre-order placement from the center.  The center meets its children at
    // both endpoints; any other edge at its new (lower) endpoint only.
    int n_slots = 0;
    auto place = [&](auto&& self, int s) -> void {
        const int e = H.edge[s];
        int cand[TM_MAX_L], nc = 0;
        for (int p = 0; p < mo->l; ++p) {
            if (!in_tree[p] || H.slot_of_edge[p] != -1) continue;  // placed or reserved
            const bool at_src = s == 0 ? (mo->src[p] == mo->src[e] || mo->dst[p] == mo->src[e])
                                       : false;
            const bool at_dst = s == 0 ? (mo->src[p] == mo->dst[e] || mo->dst[p] == mo->dst[e])
                                       : false;
            const bool at_low = s != 0 && (mo->src[p] == H.new_vertex[s] || mo->dst[p] == H.new_vertex[s]);
            if (at_src || at_dst || at_low) cand[nc++] = p;
        }
        for (int j = 0; j < nc; ++j) H.slot_of_edge[cand[j]] = -2;  // reserved
        for (int j = 0; j < nc; ++j) {
            const int p = cand[j];
            const int c = n_slots++;
            H.edge[c] = p;
            H.slot_of_edge[p] = c;
            H.parent[c] = s;
            int z;
            if (s == 0) z = (mo->src[p] == mo->src[e] || mo->dst[p] == mo->src[e]) ? mo->src[e] : mo->dst[e];
            else z = H.new_vertex[s];
            H.side[c] = z == mo->src[e] ? 0 : 1;
            H.alpha[c] = mo->src[p] == z ? +1 : -1;
            H.beta[c] = earlier(p, e) ? -1 : (earlier(e, p) ? +1 : 0);
            H.new_vertex[c] = mo->src[p] == z ? mo->dst[p] : mo->src[p];
            H.children[s][H.n_children[s]++] = c;
            self(self, c);
        }
    };
    H.edge[0] = tr->center;
    H.slot_of_edge[tr->center] = 0;
    H.parent[0] = -1;
    H.side[0] = 0;
    H.alpha[0] = 0;
    H.beta[0] = 0;
    H.new_vertex[0] = -1;
    n_slots = 1;
    place(place, 0);
    if (n_slots != H.nt) return tm_fail(TM_EINVAL, "tree: not connected through its center");
    // heights, children before parents: slots are in pre-order, so walk back
    for (int s = H.nt - 1; s >= 0; --s) {
        int h = 0;
        for (int j = 0; j < H.n_children[s]; ++j) h = std::max(h, 1 + H.height[H.children[s][j]]);
        H.height[s] = h;
    }
    H.H = H.height[0];
    for (int s = 0; s < H.nt; ++s)
        H.same_window[s] = s > 1 && H.parent[s] == H.parent[s - 1] && H.side[s] == H.side[s - 1] &&
                           H.alpha[s] == H.alpha[s - 1] && H.beta[s] == H.beta[s - 1];
    H.root_dir = H.n_children[0] > 0 ? 1 : 0;
    for (int j = 0; j < H.n_children[0]; ++j)
        if (H.side[H.children[0][j]] == 0) H.root_dir = 0;
    int r = 0;
    for (int p = 0; p < mo->l; ++p)
        if (H.slot_of_edge[p] >= 0) H.by_pi[r++] = H.slot_of_edge[p];
    // non-tree edges and their runs between tree positions
    H.n_free = 0;
    H.n_runs = 0;
    int last_tree_slot = -1;
    for (int p = 0; p < mo->l;) {
        if (H.slot_of_edge[p] >= 0) {
            last_tree_slot = H.slot_of_edge[p];
            ++p;
            continue;
        }
        const int first = H.n_free;
        while (p < mo->l && H.slot_of_edge[p] < 0) {
            H.free_src[H.n_free] = mo->src[p];
            H.free_dst[H.n_free] = mo->dst[p];
            ++H.n_free;
            ++p;
        }
        H.run_first[H.n_runs] = first;
        H.run_len[H.n_runs] = H.n_free - first;
        H.run_prev[H.n_runs] = last_tree_slot;
        H.run_next[H.n_runs] = p < mo->l ? H.slot_of_edge[p] : -1;
        ++H.n_runs;
    }
    if (H.po) {
        int free_edge[TM_MAX_L], nf = 0;
        for (int p = 0; p < mo->l; ++p)
            if (H.slot_of_edge[p] < 0) free_edge[nf++] = p;
        for (int s = 0; s < kMaxSlots; ++s) H.po_tpred[s] = 0;
        for (int s = 0; s < H.nt; ++s)
            for (int s2 = 0; s2 < H.nt; ++s2)
                if (earlier(H.edge[s2], H.edge[s])) H.po_tpred[s] |= (uint16_t)(1u << s2);
        for (int f = 0; f < TM_MAX_L; ++f) {
            H.po_f_tpred[f] = H.po_f_tsucc[f] = H.po_f_fpred[f] = 0;
            if (f >= nf) continue;
            for (int s = 0; s < H.nt; ++s) {
                if (earlier(H.edge[s], free_edge[f])) H.po_f_tpred[f] |= (uint16_t)(1u << s);
                if (earlier(free_edge[f], H.edge[s])) H.po_f_tsucc[f] |= (uint16_t)(1u << s);
            }
            for (int f2 = 0; f2 < nf; ++f2)
                if (earlier(free_edge[f2], free_edge[f])) H.po_f_fpred[f] |= (uint16_t)(1u << f2);
        }
    }
    return TM_OK;
}

extern "C" int tm_default_tree(const tm_motif* mo, tm_tree* out) {
    TM_TRY(motif_check(mo));
    if (!out) return tm_fail(TM_EINVAL, "tree: NULL output");
    const int need = mo->k - 1;
    long best_loose = -1;
    int32_t best[8] = {0};
    for (uint32_t mask = 0; mask < (1u << mo->l); ++mask) {
        if (__builtin_popcount(mask) != need) continue;
        int32_t e[8];
        int c = 0;
        for (int p = 0; p < mo->l; ++p)
            if (mask >> p & 1) e[c++] = p;
        if (!spanning_tree_of(mo, e, c)) continue;
        long loose = 0;
        for (int x = 0; x < mo->k; ++x) {
            int inc[8], ni = 0;
            for (int j = 0; j < c; ++j)
                if (mo->src[e[j]] == x || mo->dst[e[j]] == x) inc[ni++] = e[j];
            for (int a = 0; a < ni; ++a)
                for (int b = a + 1; b < ni; ++b) loose += std::abs(inc[a] - inc[b]) - 1;
        }
        const bool better = best_loose < 0 || loose < best_loose ||
                            (loose == best_loose && std::lexicographical_compare(e, e + c, best, best + c));
        if (better) {
            best_loose = loose;
            std::memcpy(best, e, sizeof(int32_t) * c);
        }
    }
    if (best_loose < 0) return tm_fail(TM_EINVAL, "motif: no spanning tree");
    tm_tree t;
    std::memset(&t, 0, sizeof t);
    t.n_edges = need;
    std::memcpy(t.edge, best, sizeof(int32_t) * need);
    int best_h = 1 << 30;
    int center = best[0];
    for (int j = 0; j < need; ++j) {  // best[] is increasing: ties keep the smaller index
        t.center = best[j];
        HostPlan P;
        TM_TRY(plan_build(mo, &t, &P));
        if (P.H < best_h) {
            best_h = P.H;
            center = best[j];
        }
    }
    t.center = center;
    *out = t;
    return TM_OK;
}

// ---------------------------------------------------------------------------
// Entry points.
// ---------------------------------------------------------------------------
extern "C" const char* tm_strerror(int code) {
    switch (code) {
        case TM_OK: return "ok";
        case TM_EINVAL: return "invalid argument";
        case TM_ESELFLOOP: return "self loop in the graph";
        case TM_EDUP: return "duplicate (u, v, t) tuple";
        case TM_EOVERFLOW: return "count reaches 2^128";
        case TM_ERANGE: return "value outside the supported range";
        case TM_ENOMEM: return "out of device memory";
        case TM_EDEVICE: return "HIP runtime error";
        case TM_EADMIT: return "query exceeds the server's memory budget";
        case TM_EAGAIN: return "query not finished";
        case TM_ECANCELED: return "server stopped before the query finished";
        default: return "unknown error";
    }
}

extern "C" const char* tm_last_error(void) { return g_last_error; }

static hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

extern "C" int tm_graph_create(const int32_t* src, const int32_t* dst, const int64_t* t, int64_t m,
                               int32_t n, int ptr_kind, const tm_allocator* alloc, void* stream,
                               tm_graph** out) {
    if (!out) return tm_fail(TM_EINVAL, "graph: NULL output");
    if (m < 0 || m >= ((int64_t)1 << 31) || n < 0 || n == INT32_MAX)
        return tm_fail(TM_EINVAL, "graph: m = %lld or n = %d out of range", (long long)m, n);
    if (m > 0 && (!src || !dst || !t)) return tm_fail(TM_EINVAL, "graph: NULL edge array");
    if (ptr_kind != TM_PTR_HOST && ptr_kind != TM_PTR_DEVICE)
        return tm_fail(TM_EINVAL, "graph: bad ptr_kind %d", ptr_kind);
    hipStream_t st = as_stream(stream);
    tm_graph* g = new (std::nothrow) tm_graph();
    if (!g) return tm_fail(TM_ENOMEM, "graph: host allocation");
    g->m = m;
    g->n = n;
    if (alloc) {
        if (!alloc->alloc || !alloc->free) {
            delete g;
            return tm_fail(TM_EINVAL, "graph: allocator without alloc or free");
        }
        g->alloc = *alloc;
        g->has_alloc = true;
    }
    AllocScope scope_(alloc_of(g));
    (void)hipGetDevice(&g->device);
    g->arena.stream = st;
    const int32_t *ds = src, *dd = dst;
    const int64_t* dt = t;
    void* staged[3] = {nullptr, nullptr, nullptr};
    int rc = TM_OK;
    if (ptr_kind == TM_PTR_HOST && m > 0) {
        const size_t sz[3] = {m * sizeof(int32_t), m * sizeof(int32_t), m * sizeof(int64_t)};
        const void* hp[3] = {src, dst, t};
        for (int a = 0; a < 3 && rc == TM_OK; ++a) {
            hipError_t e = dev_alloc(&staged[a], sz[a], st);
            if (e == hipSuccess) e = hipMemcpyAsync(staged[a], hp[a], sz[a], hipMemcpyHostToDevice, st);
            if (e != hipSuccess)
                rc = tm_fail(e == hipErrorOutOfMemory ? TM_ENOMEM : TM_EDEVICE, "graph: staging: %s",
                             hipGetErrorString(e));
        }
        ds = static_cast<const int32_t*>(staged[0]);
        dd = static_cast<const int32_t*>(staged[1]);
        dt = static_cast<const int64_t*>(staged[2]);
    }
    if (rc == TM_OK) rc = graph_build(g, ds, dd, dt, st);
    for (void* p : staged)
        if (p) (void)dev_free(p, st);
    (void)sync_stream(st);
    if (rc != TM_OK) {
        g->arena.release();
        delete g;
        return rc;
    }
    *out = g;
    return TM_OK;
}

extern "C" void tm_graph_destroy(tm_graph* g) {
    if (!g) return;
    g->arena.release();
    delete g;
}

extern "C" int tm_graph_info(const tm_graph* g, int64_t* m, int32_t* n, int64_t* t_shift,
                             int64_t* t_span, uint64_t* device_bytes) {
    if (!g) return tm_fail(TM_EINVAL, "graph: NULL");
    if (m) *m = g->m;
    if (n) *n = g->n;
    if (t_shift) *t_shift = g->shift;
    if (t_span) *t_span = g->T;
    if (device_bytes) *device_bytes = g->arena.bytes;
    return TM_OK;
}

extern "C" int tm_graph_export(const tm_graph* g, int which, void* host_out, void* stream) {
    AllocScope scope_(alloc_of(g));
    if (!g || !host_out) return tm_fail(TM_EINVAL, "graph_export: NULL");
    const DevGraph& D = g->d;
    const void* p = nullptr;
    size_t bytes = 0;
    const size_t m = (size_t)g->m, n1 = (size_t)g->n + 1;
    switch (which) {
        case TM_ARR_SRC: p = D.src; bytes = m * 4; break;
        case TM_ARR_DST: p = D.dst; bytes = m * 4; break;
        case TM_ARR_T: p = D.t; bytes = m * 8; break;
        case TM_ARR_OUT_OFF: p = D.off[0]; bytes = n1 * 4; break;
        case TM_ARR_IN_OFF: p = D.off[1]; bytes = n1 * 4; break;
        case TM_ARR_OUT_EID: p = D.leid[0]; bytes = m * 4; break;
        case TM_ARR_IN_EID: p = D.leid[1]; bytes = m * 4; break;
        case TM_ARR_OUTN_EID: p = D.neid[0]; bytes = m * 4; break;
        case TM_ARR_INN_EID: p = D.neid[1]; bytes = m * 4; break;
        case TM_ARR_OUT_T:
        case TM_ARR_IN_T: {
            const int dir = which == TM_ARR_IN_T ? 1 : 0;
            if (!D.lt32[dir]) {
                p = D.lt[dir];
                bytes = m * 8;
                break;
            }
            // 32-bit lists: widened on the host
            if (m == 0) return TM_OK;
            std::vector<uint32_t> h32(m);
            hipStream_t st = as_stream(stream);
            TM_HIP(hipMemcpyAsync(h32.data(), D.lt32[dir], m * 4, hipMemcpyDeviceToHost, st));
            TM_HIP(sync_stream(st));
            int64_t* out = static_cast<int64_t*>(host_out);
            for (size_t i = 0; i < m; ++i) out[i] = (int64_t)h32[i];
            return TM_OK;
        }
        case TM_ARR_OUT_NBR:
        case TM_ARR_IN_NBR: {
            const int dir = which == TM_ARR_IN_NBR ? 1 : 0;
            if (!D.lnt[dir]) {
                p = D.lnbr[dir];
                bytes = m * 4;
                break;
            }
            // (neighbour, time) records: the neighbours taken out on the host
            if (m == 0) return TM_OK;
            std::vector<uint2> hnt(m);
            hipStream_t st = as_stream(stream);
            TM_HIP(hipMemcpyAsync(hnt.data(), D.lnt[dir], m * sizeof(uint2), hipMemcpyDeviceToHost, st));
            TM_HIP(sync_stream(st));
            int32_t* out = static_cast<int32_t*>(host_out);
            for (size_t i = 0; i < m; ++i) out[i] = (int32_t)hnt[i].x;
            return TM_OK;
        }
        case TM_ARR_OUT_POS: p = D.tpos[0]; bytes = m * 4; break;
        case TM_ARR_IN_POS: p = D.tpos[1]; bytes = m * 4; break;
        case TM_ARR_OUTN_KEY: p = D.nkey[0]; bytes = m * 8; break;
        case TM_ARR_INN_KEY: p = D.nkey[1]; bytes = m * 8; break;
        case TM_ARR_OUTN_POS: p = D.nxref[0]; bytes = m * 4; break;
        case TM_ARR_INN_POS: p = D.nxref[1]; bytes = m * 4; break;
        default: return tm_fail(TM_EINVAL, "graph_export: unknown array %d", which);
    }
    if (bytes == 0 || !p) return TM_OK;
    hipStream_t st = as_stream(stream);
    TM_HIP(hipMemcpyAsync(host_out, p, bytes, hipMemcpyDeviceToHost, st));
    TM_HIP(sync_stream(st));
    return TM_OK;
}

// ---------------------------------------------------------------------------
// Choosing the spanning tree (Sec. "Choosing the Spanning Tree", Alg. 7 and 8).
// ---------------------------------------------------------------------------
namespace {
struct TreeCand {
    long loose;
    int32_t e[8];
    int c;
    int H;
    int center;
};

// Every (spanning tree, center) pair with its constraint looseness (per motif
// vertex, over unordered pairs of tree edges incident to it, |pi(e1) - pi(e2)| - 1)
// and rooted height; ordered by looseness, then edge set, height and center.
int tree_cands(const tm_motif* mo, std::vector<TreeCand>& out) {
    out.clear();
    const int need = mo->k - 1;
    for (uint32_t mask = 0; mask < (1u << mo->l); ++mask) {
        if (__builtin_popcount(mask) != need) continue;
        TreeCand t;
        t.c = 0;
        for (int p = 0; p < mo->l; ++p)
            if (mask >> p & 1) t.e[t.c++] = p;
        if (!spanning_tree_of(mo, t.e, t.c)) continue;
        t.loose = 0;
        for (int x = 0; x < mo->k; ++x) {
            int inc[8], ni = 0;
            for (int j = 0; j < t.c; ++j)
                if (mo->src[t.e[j]] == x || mo->dst[t.e[j]] == x) inc[ni++] = t.e[j];
            for (int a = 0; a < ni; ++a)
                for (int b = a + 1; b < ni; ++b) t.loose += std::abs(inc[a] - inc[b]) - 1;
        }
        for (int j = 0; j < t.c; ++j) {
            tm_tree tr;
            std::memset(&tr, 0, sizeof tr);
            tr.n_edges = t.c;
            std::memcpy(tr.edge, t.e, sizeof(int32_t) * t.c);
            tr.center = t.e[j];
            HostPlan P;
            TM_TRY(plan_build(mo, &tr, &P));
            TreeCand u = t;
            u.center = t.e[j];
            u.H = P.H;
            out.push_back(u);
        }
    }
    std::stable_sort(out.begin(), out.end(), [](const TreeCand& a, const TreeCand& b) {
        if (a.loose != b.loose) return a.loose < b.loose;
        if (!std::equal(a.e, a.e + a.c, b.e)) return std::lexicographical_compare(a.e, a.e + a.c, b.e, b.e + b.c);
        if (a.H != b.H) return a.H < b.H;
        return a.center < b.center;
    });
    return TM_OK;
}

tm_tree to_tree(const TreeCand& t) {
    tm_tree tr;
    std::memset(&tr, 0, sizeof tr);
    tr.n_edges = t.c;
    std::memcpy(tr.edge, t.e, sizeof(int32_t) * t.c);
    tr.center = t.center;
    return tr;
}
}  // namespace

extern "C" int tm_tree_candidates(const tm_motif* mo, tm_tree* out, int64_t* looseness, int max_out, int* n_out) {
    TM_TRY(motif_check(mo));
    if (max_out < 0 || (max_out > 0 && !out) || !n_out) return tm_fail(TM_EINVAL, "tree_candidates: bad arguments");
    std::vector<TreeCand> c;
    TM_TRY(tree_cands(mo, c));
    *n_out = (int)c.size();
    for (int x = 0; x < max_out && x < (int)c.size(); ++x) {
        out[x] = to_tree(c[x]);
        if (looseness) looseness[x] = c[x].loose;
    }
    return TM_OK;
}

extern "C" int tm_choose_tree(tm_graph* g, const tm_motif* mo, int n_c, void* stream, tm_tree* best,
                              tm_u128* W_out, int* n_eval) {
    AllocScope scope_(alloc_of(g));
    if (!g || !best || n_c < 1) return tm_fail(TM_EINVAL, "choose_tree: bad arguments");
    TM_TRY(motif_check(mo));
    std::vector<TreeCand> c;
    TM_TRY(tree_cands(mo, c));
    const int n = std::min<int>(n_c, (int)c.size());
    int arg = -1;
    u128 bestW = 0;
    for (int x = 0; x < n; ++x) {
        const tm_tree tr = to_tree(c[x]);
        tm_weights* w = nullptr;
        TM_TRY(tm_weights_create(g, mo, &tr, stream, &w));
        const u128 W = w->W;
        tm_weights_destroy(w);
        if (W_out) {
            W_out[x].lo = (u64)W;
            W_out[x].hi = (u64)(W >> 64);
        }
        if (arg < 0 || W < bestW) {
            arg = x;
            bestW = W;
        }
    }
    *best = to_tree(c[arg]);
    if (n_eval) *n_eval = n;
    return TM_OK;
}

extern "C" int tm_weights_create(tm_graph* g, const tm_motif* mo, const tm_tree* tr, void* stream,
                                 tm_weights** out) {
    return tm_weights_create_ex(g, mo, tr, TM_C_ALL, stream, out);
}

namespace {

int weights_create(tm_graph* g, const tm_motif* mo, const tm_tree* tr, uint32_t constraints, void* stream,
                   tm_weights** out, u64* model_bytes) {
    if (!g || !out) return tm_fail(TM_EINVAL, "weights: NULL argument");
    if (constraints & ~(uint32_t)TM_C_ALL) return tm_fail(TM_EINVAL, "weights: constraints %u", constraints);
    TM_TRY(motif_check(mo));
    tm_tree def;
    if (!tr) {
        TM_TRY(tm_default_tree(mo, &def));
        tr = &def;
    }
    tm_weights* w = new (std::nothrow) tm_weights();
    if (!w) return tm_fail(TM_ENOMEM, "weights: host allocation");
    w->g = g;
    w->arena.stream = as_stream(stream);
    w->constraints = constraints;
    int rc = plan_build(mo, tr, &w->plan);
    if (rc == TM_OK) rc = weights_build(w, as_stream(stream), model_bytes);
    if (rc != TM_OK) {
        w->arena.release();
        delete w;
        return rc;
    }
    *out = w;
    return TM_OK;
}

}  // namespace

extern "C" int tm_weights_create_ex(tm_graph* g, const tm_motif* mo, const tm_tree* tr, uint32_t constraints,
                                    void* stream, tm_weights** out) {
    AllocScope scope_(alloc_of(g));
    return weights_create(g, mo, tr, constraints, stream, out, nullptr);
}

extern "C" int tm_weights_model_bytes(tm_graph* g, const tm_motif* mo, const tm_tree* tr, void* stream,
                                      uint64_t* bytes) {
    AllocScope scope_(alloc_of(g));
    if (!bytes) return tm_fail(TM_EINVAL, "weights_model_bytes: NULL argument");
    // the counting pass is not a timed stage
    const bool was = prof_suspended();
    prof_suspend(true);
    tm_weights* w = nullptr;
    u64 b = 0;
    const int rc = weights_create(g, mo, tr, TM_C_ALL, stream, &w, &b);
    prof_suspend(was);
    if (rc != TM_OK) return rc;
    tm_weights_destroy(w);
    *bytes = b;
    return TM_OK;
}

extern "C" int tm_weights_footprint(const tm_graph* g, const tm_motif* mo, const tm_tree* tr,
                                    int32_t wide, uint64_t* bytes) {
    if (!g || !bytes) return tm_fail(TM_EINVAL, "weights_footprint: NULL argument");
    TM_TRY(motif_check(mo));
    tm_tree def;
    if (!tr) {
        TM_TRY(tm_default_tree(mo, &def));
        tr = &def;
    }
    HostPlan P;
    TM_TRY(plan_build(mo, tr, &P));
    const int64_t q = g->m > 0 ? g->T / mo->delta + 1 : 0;
    *bytes = weights_footprint(P, g->m, q, wide != 0);
    return TM_OK;
}

extern "C" void tm_weights_destroy(tm_weights* w) {
    if (!w) return;
    w->arena.release();
    delete w;
}

extern "C" int tm_weights_info(const tm_weights* w, tm_u128* W, int64_t* q, int32_t* wide,
                               uint64_t* device_bytes, tm_tree* tree) {
    if (!w) return tm_fail(TM_EINVAL, "weights: NULL");
    if (W) {
        W->lo = (u64)w->W;
        W->hi = (u64)(w->W >> 64);
    }
    if (q) *q = w->q;
    if (wide) *wide = w->wide ? 1 : 0;
    if (device_bytes) *device_bytes = w->arena.bytes;
    if (tree) *tree = w->plan.tree;
    return TM_OK;
}

extern "C" int tm_weights_export(const tm_weights* w, int32_t s, int32_t slot, tm_u128* host_out,
                                 void* stream) {
    AllocScope scope_(w ? alloc_of(w->g) : nullptr);
    if (!w || !host_out) return tm_fail(TM_EINVAL, "weights_export: NULL");
    const HostPlan& P = w->plan;
    if (s < 0 || s >= P.mo.l || P.slot_of_edge[s] < 0 || slot < 0 || slot > 1)
        return tm_fail(TM_EINVAL, "weights_export: edge %d / slot %d", s, slot);
    const int sl = P.slot_of_edge[s];
    const int64_t m = w->g->m;
    if (m == 0) return TM_OK;
    hipStream_t st = as_stream(stream);
    std::vector<int64_t> t(m);
    TM_HIP(hipMemcpyAsync(t.data(), w->g->d.t, m * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    const bool leaf = P.n_children[sl] == 0;
    // the center's tables follow the set's width, a list table its own
    const bool twide = sl == 0 ? w->wide : w->list_wide;
    const size_t wsz = twide ? 16 : 8;
    // values are differences of neighbouring prefix entries: along eid order
    // for the center, along the T order of the slot's list otherwise
    std::vector<unsigned char> pre[2];
    std::vector<int32_t> pos;
    const int dir = P.alpha[sl] > 0 ? 0 : 1;
    if (!leaf) {
        for (int par = 0; par < 2; ++par) {
            pre[par].resize((m + 1) * wsz);
            const void* src = sl == 0 ? w->qc[par] : w->qt[sl][par];
            TM_HIP(hipMemcpyAsync(pre[par].data(), src, (m + 1) * wsz, hipMemcpyDeviceToHost, st));
        }
        if (sl != 0) {
            pos.resize(m);
            TM_HIP(hipMemcpyAsync(pos.data(), w->g->d.tpos[dir], m * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        }
    }
    TM_HIP(sync_stream(st));
    auto at = [&](int par, int64_t p) {
        const unsigned char* b = pre[par].data() + p * wsz;
        u64 lo = 0, hi = 0;
        std::memcpy(&lo, b, 8);
        if (twide) std::memcpy(&hi, b + 8, 8);
        const u128 v = ((u128)hi << 64) | lo;
        return twide ? v : (u128)(u64)v;
    };
    for (int64_t e = 0; e < m; ++e) {
        const int64_t i = t[e] / w->ilen - slot;
        tm_u128 x = {0, 0};
        if (i >= 0 && i < w->q) {
            if (leaf) {
                x.lo = 1;
            } else {
                const int par = (int)(i & 1);
                const int64_t p = sl == 0 ? e : pos[e];
                u128 d = at(par, p + 1) - at(par, p);
                if (!twide) d = (u64)d;
                x.lo = (u64)d;
                x.hi = (u64)(d >> 64);
            }
        }
        host_out[e] = x;
    }
    return TM_OK;
}

extern "C" int tm_weights_intervals(const tm_weights* w, tm_u128* host_out, void* stream) {
    AllocScope scope_(w ? alloc_of(w->g) : nullptr);
    if (!w || !host_out) return tm_fail(TM_EINVAL, "weights_intervals: NULL");
    if (w->q == 0) return TM_OK;
    hipStream_t st = as_stream(stream);
    const size_t wsz = w->wide ? 16 : 8;
    std::vector<unsigned char> c((w->q + 1) * wsz);
    TM_HIP(hipMemcpyAsync(c.data(), w->cumW, c.size(), hipMemcpyDeviceToHost, st));
    TM_HIP(sync_stream(st));
    auto at = [&](int64_t i) {
        u128 x = 0;
        u64 lo = 0, hi = 0;
        std::memcpy(&lo, c.data() + i * wsz, 8);
        if (w->wide) std::memcpy(&hi, c.data() + i * wsz + 8, 8);
        x = ((u128)hi << 64) | lo;
        return x;
    };
    for (int64_t i = 0; i < w->q; ++i) {
        const u128 d = at(i + 1) - at(i);
        host_out[i].lo = (u64)d;
        host_out[i].hi = (u64)(d >> 64);
    }
    return TM_OK;
}

static double u128_to_double(tm_u128 x) { return (double)(((u128)x.hi << 64) | x.lo); }

// Unsigned 256-bit value as (hi, lo) 128-bit halves.
struct U256 {
    u128 hi, lo;
};

// Full 128 x 128 -> 256-bit product from four 64 x 64 -> 128 partial products.
static U256 mul_wide(u128 a, u128 b) {
    const u64 a0 = (u64)a, a1 = (u64)(a >> 64), b0 = (u64)b, b1 = (u64)(b >> 64);
    const u128 p00 = (u128)a0 * b0, p01 = (u128)a0 * b1, p10 = (u128)a1 * b0, p11 = (u128)a1 * b1;
    // middle column: high half of p00 plus the low halves of the cross terms
    const u128 mid = (p00 >> 64) + (u64)p01 + (u64)p10;
    U256 r;
    r.lo = (mid << 64) | (u64)p00;
    r.hi = p11 + (p01 >> 64) + (p10 >> 64) + (mid >> 64);
    return r;
}

// Nearest double to a 256-bit value (ties to even): shifted down to 128
// bits with the shifted-out bits folded into bit 0 (they lie far below the
// 53-bit rounding position, so only whether any was set matters), converted
// by the compiler's correctly rounded u128 conversion, then scaled back by
// an exact power of two.
static double u256_to_double(U256 x) {
    if (x.hi == 0) return (double)x.lo;
    const u64 hh = (u64)(x.hi >> 64), hl = (u64)x.hi;
    const int top = hh ? 255 - __builtin_clzll(hh) : 191 - __builtin_clzll(hl);  // top set bit
    const int sh = top - 127;                                                     // 1 .. 128
    const u128 low_mask = sh == 128 ? ~(u128)0 : (((u128)1 << sh) - 1);
    const bool sticky = (x.lo & low_mask) != 0;
    const u128 v = sh == 128 ? x.hi : ((x.hi << (128 - sh)) | (x.lo >> sh));
    return __builtin_ldexp((double)(v | (sticky ? 1 : 0)), sh);
}

// The estimate (Alg. 6) and its standard error (Sec. 4.4, Lemma
// "unbiased-estimate": the estimate is W / 2 times the mean of the terms
// Y = 2 M_phi / N_phi, so its standard error is (W / 2) s / sqrt(k) with s^2
// the unbiased sample variance).  s^2 = D / (k (k - 1)) with
// D = k sum Y^2 - (sum Y)^2, formed exactly in 256 bits from the exact sums
// and rounded once; 0 when k < 2, W = 0 or the sum of squares saturated.
void finish_result(tm_result* r) {
    const double W = u128_to_double(r->W);
    const double acc2 = u128_to_double(r->acc2);
    const double k = (double)r->k;
    r->estimate = r->k ? W * (acc2 / (2.0 * k)) : 0.0;
    r->std_error = 0.0;
    const u128 Wx = ((u128)r->W.hi << 64) | r->W.lo;
    if (r->k < 2 || Wx == 0 || (r->flags & TM_F_SQ_SATURATED)) return;
    const u128 s1 = ((u128)r->acc2.hi << 64) | r->acc2.lo;
    const u128 s2 = ((u128)r->acc2_sq.hi << 64) | r->acc2_sq.lo;
    const U256 a = mul_wide((u128)r->k, s2), b = mul_wide(s1, s1);
    if (a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo)) return;  // not for sums over at most k samples
    U256 D;
    D.lo = a.lo - b.lo;
    D.hi = a.hi - b.hi - (a.lo < b.lo ? 1 : 0);
    const double Dd = u256_to_double(D);
    const double km1 = (double)(r->k - 1);
    const double var = Dd / (k * km1);
    r->std_error = (W / 2.0) * __builtin_sqrt(var / k);
}

extern "C" int tm_result_finish(tm_result* r) {
    if (!r) return tm_fail(TM_EINVAL, "result_finish: NULL");
    finish_result(r);
    return TM_OK;
}

extern "C" int tm_sample(tm_weights* w, uint64_t seed, uint64_t j0, uint64_t count,
                         uint64_t k_total, void* stream, tm_result* out, tm_sample_rec* recs) {
    AllocScope scope_(w ? alloc_of(w->g) : nullptr);
    if (!w || !out) return tm_fail(TM_EINVAL, "sample: NULL argument");
    if (count > 0 && j0 + count < j0) return tm_fail(TM_EINVAL, "sample: id range wraps");
    TM_TRY(sample_run(w, seed, j0, count, k_total, as_stream(stream), out, recs, nullptr));
    finish_result(out);
    out->status = TM_OK;
    return TM_OK;
}

extern "C" int tm_sample_noalloc(tm_weights* w, uint64_t seed, uint64_t j0, uint64_t count, uint64_t k_total,
                                 void* stream, tm_result* out, tm_sample_rec* recs) {
    if (!w || !out) return tm_fail(TM_EINVAL, "sample_noalloc: NULL argument");
    if (count > 0 && j0 + count < j0) return tm_fail(TM_EINVAL, "sample_noalloc: id range wraps");
    TM_TRY(sample_run_noalloc(w, seed, j0, count, k_total, as_stream(stream), out, recs));
    finish_result(out);
    out->status = TM_OK;
    return TM_OK;
}

extern "C" int tm_sample_model_bytes(tm_weights* w, uint64_t seed, uint64_t j0, uint64_t count,
                                     void* stream, uint64_t* bytes) {
    AllocScope scope_(w ? alloc_of(w->g) : nullptr);
    if (!w || !bytes) return tm_fail(TM_EINVAL, "sample_model_bytes: NULL argument");
    tm_result r;
    return sample_run(w, seed, j0, count, count, as_stream(stream), &r, nullptr,
                      reinterpret_cast<u64*>(bytes));
}

extern "C" int tm_estimate(tm_graph* g, const tm_motif* mo, const tm_tree* tr, uint64_t k,
                           uint64_t seed, void* stream, tm_result* out, tm_sample_rec* recs) {
    return tm_estimate_ex(g, mo, tr, TM_C_ALL, k, seed, stream, out, recs);
}

namespace {

// The 64-bit weight build and the sampling enqueued together with one
// synchronisation at the end (graphs below 2^23 edges, where a synchronous
// build checks for overflow only at its end anyway).  *done is false when
// the 64-bit tables overflowed: the caller then runs the synchronous path.
int estimate_enqueued(tm_graph* g, const tm_motif* mo, const tm_tree* tr, uint32_t constraints, u64 k, u64 seed,
                      hipStream_t st, tm_result* out, bool* done) {
    *done = false;
    if (constraints & ~(uint32_t)TM_C_ALL) return tm_fail(TM_EINVAL, "weights: constraints %u", constraints);
    TM_TRY(motif_check(mo));
    tm_tree def;
    if (!tr) {
        TM_TRY(tm_default_tree(mo, &def));
        tr = &def;
    }
    tm_weights* w = new (std::nothrow) tm_weights();
    if (!w) return tm_fail(TM_ENOMEM, "weights: host allocation");
    w->g = g;
    w->arena.stream = st;
    w->constraints = constraints;
    int* flag = nullptr;
    int rc = plan_build(mo, tr, &w->plan);
    if (rc == TM_OK && dev_alloc((void**)&flag, sizeof(int), st) != hipSuccess)
        rc = tm_fail(TM_ENOMEM, "estimate: device allocation");
    if (rc == TM_OK) rc = fill_u32(flag, 1, 0u, st);
    StageTimer tw;
    std::vector<std::unique_ptr<StageTimer>> levels;
    if (rc == TM_OK) {
        tw.start(TM_STAGE_WEIGHTS, st);
        rc = weights_enqueue(w, st, flag, &levels);
        tw.stop();
    }
    bool overflowed = false;
    if (rc == TM_OK) rc = sample_run(w, seed, 0, k, k, st, out, nullptr, nullptr, flag, &overflowed);
    // sample_run synchronised the stream (on success)
    if (sync_stream(st) != hipSuccess && rc == TM_OK) rc = tm_fail(TM_EDEVICE, "estimate: synchronise");
    tw.finish();
    for (auto& t : levels) t->finish();
    if (flag) (void)dev_free(flag, st);
    tm_weights_destroy(w);
    if (rc == TM_OK) *done = !overflowed;
    return rc;
}

}  // namespace

extern "C" int tm_estimate_ex(tm_graph* g, const tm_motif* mo, const tm_tree* tr, uint32_t constraints,
                              uint64_t k, uint64_t seed, void* stream, tm_result* out, tm_sample_rec* recs) {
    AllocScope scope_(alloc_of(g));
    if (!out) return tm_fail(TM_EINVAL, "estimate: NULL output");
    // records need W on the host first (a W = 0 run writes "not drawn"
    // records): they take the synchronous path
    if (g && k > 0 && g->m > 0 && g->m < ((int64_t)1 << 23) && !recs) {
        bool done = false;
        TM_TRY(estimate_enqueued(g, mo, tr, constraints, k, seed, as_stream(stream), out, &done));
        if (done) {
            finish_result(out);
            out->status = TM_OK;
            return TM_OK;
        }
    }
    tm_weights* w = nullptr;
    TM_TRY(tm_weights_create_ex(g, mo, tr, constraints, stream, &w));
    const int rc = tm_sample(w, seed, 0, k, k, stream, out, recs);
    tm_weights_destroy(w);
    return rc;
}

// ---------------------------------------------------------------------------
// Batched estimation.
// ---------------------------------------------------------------------------
static std::mutex g_cfg_mu;

extern "C" int tm_batch_config(int tile, int blocks, int* prev_tile, int* prev_blocks) {
    if (tile < 256 || blocks < 0) return tm_fail(TM_EINVAL, "batch_config: tile %d, blocks %d", tile, blocks);
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    if (prev_tile) *prev_tile = g_batch_config.tile;
    if (prev_blocks) *prev_blocks = g_batch_config.blocks;
    g_batch_config.tile = tile;
    g_batch_config.blocks = blocks;
    return TM_OK;
}

extern "C" int tm_batch_options(const tm_batch_opts* in, tm_batch_opts* prev) {
    if (in && (in->tile < 256 || in->blocks < 0 || in->root_lds < 0 || in->root_lds > 65536))
        return tm_fail(TM_EINVAL, "batch_options: tile %d, blocks %d, root_lds %d", in->tile, in->blocks,
                       in->root_lds);
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    if (prev) {
        prev->tile = g_batch_config.tile;
        prev->blocks = g_batch_config.blocks;
        prev->root_lds = g_batch_config.root_lds;
        prev->pad = 0;
        prev->group_limit = g_batch_config.group_limit;
    }
    if (in) {
        g_batch_config.tile = in->tile;
        g_batch_config.blocks = in->blocks;
        g_batch_config.root_lds = in->root_lds;
        g_batch_config.group_limit = in->group_limit;
    }
    return TM_OK;
}

BatchConfig batch_config_now() {
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    return g_batch_config;
}

// Results of k[i] samples (ids 0 .. k[i] - 1) of every job, in one batched pass.
int sample_batch_results(tm_weights* const* w, const uint64_t* k, const uint64_t* seed, int n_jobs,
                         hipStream_t st, tm_result* out) {
    std::vector<u64> j0(n_jobs, 0), kk(k, k + n_jobs), ss(seed, seed + n_jobs);
    std::vector<JobSums> sums(n_jobs);
    TM_TRY(batch_sample_pass(w, j0.data(), kk.data(), ss.data(), n_jobs, st, sums.data(), batch_config_now()));
    for (int i = 0; i < n_jobs; ++i) {
        tm_result& o = out[i];
        std::memset(&o, 0, sizeof o);
        o.k = kk[i];
        o.q = w[i]->q;
        o.W.lo = (u64)w[i]->W;
        o.W.hi = (u64)(w[i]->W >> 64);
        if (w[i]->wide) o.flags |= TM_F_WIDE;
        if (w[i]->W == 0) o.flags |= TM_F_W_ZERO;
        sums_to_result(sums[i], &o);
        if (o.status == TM_OK) finish_result(&o);
    }
    return TM_OK;
}

extern "C" int tm_sample_batch(tm_weights* const* w, const uint64_t* k, const uint64_t* seed, int n_jobs,
                               void* stream, tm_result* out) {
    AllocScope scope_(w && n_jobs > 0 && w[0] ? alloc_of(w[0]->g) : nullptr);
    if (n_jobs < 0 || (n_jobs > 0 && (!w || !k || !seed || !out)))
        return tm_fail(TM_EINVAL, "sample_batch: bad arguments");
    for (int i = 0; i < n_jobs; ++i)
        if (!w[i]) return tm_fail(TM_EINVAL, "sample_batch: job %d has no weights", i);
    if (n_jobs == 0) return TM_OK;
    TM_TRY(sample_batch_results(w, k, seed, n_jobs, as_stream(stream), out));
    return TM_OK;
}

extern "C" int tm_estimate_batch(tm_graph* const* g, const tm_motif* mo, const tm_tree* const* tr,
                                 const uint64_t* k, const uint64_t* seed, int n_jobs, void* stream,
                                 tm_result* out) {
    AllocScope scope_(g && n_jobs > 0 ? alloc_of(g[0]) : nullptr);
    if (n_jobs < 0 || (n_jobs > 0 && (!g || !mo || !k || !seed || !out)))
        return tm_fail(TM_EINVAL, "estimate_batch: bad arguments");
    if (n_jobs == 0) return TM_OK;
    hipStream_t st = as_stream(stream);
    std::vector<tm_weights*> ws(n_jobs, nullptr);
    std::vector<int> status(n_jobs, TM_OK);
    int* flags = nullptr;
    u64* wdev = nullptr;
    TM_HIP(dev_alloc((void**)&flags, n_jobs * sizeof(int), st));
    TM_HIP(dev_alloc((void**)&wdev, n_jobs * sizeof(u64), st));
    TM_TRY(fill_u32(flags, n_jobs, 0u, st));
    TM_TRY(fill_u32(wdev, 2 * n_jobs, 0u, st));
    StageTimer timer;
    timer.start(TM_STAGE_WEIGHTS, st);
    // every job's 64-bit weight build, back to back, no synchronisation
    for (int i = 0; i < n_jobs; ++i) {
        if (!g[i]) { status[i] = tm_fail(TM_EINVAL, "estimate_batch: job %d has no graph", i); continue; }
        tm_tree def;
        const tm_tree* ti = tr ? tr[i] : nullptr;
        if (!ti) {
            const int rc = tm_default_tree(&mo[i], &def);
            if (rc != TM_OK) { status[i] = rc; continue; }
            ti = &def;
        }
        tm_weights* w = new (std::nothrow) tm_weights();
        if (!w) { status[i] = tm_fail(TM_ENOMEM, "estimate_batch: host allocation"); continue; }
        w->g = g[i];
        w->arena.stream = st;
        int rc = plan_build(&mo[i], ti, &w->plan);
        if (rc == TM_OK) rc = weights_enqueue(w, st, flags + i);
        if (rc == TM_OK && w->q > 0)
            rc = hipMemcpyAsync(wdev + i, static_cast<const unsigned char*>(w->cumW) + w->q * 8, 8,
                                hipMemcpyDeviceToDevice, st) == hipSuccess ? TM_OK : TM_EDEVICE;
        if (rc != TM_OK) {
            w->arena.release();
            delete w;
            status[i] = rc;
            continue;
        }
        ws[i] = w;
    }
    std::vector<int> hflags(n_jobs, 0);
    std::vector<u64> hW(n_jobs, 0);
    TM_HIP(read_back({{hflags.data(), flags, n_jobs * sizeof(int)}, {hW.data(), wdev, n_jobs * sizeof(u64)}}, st));
    TM_HIP(dev_free(flags, st));
    TM_HIP(dev_free(wdev, st));
    // jobs whose 64-bit build overflowed are rebuilt with the widening path
    for (int i = 0; i < n_jobs; ++i) {
        if (!ws[i]) continue;
        if (hflags[i]) {
            const int rc = weights_build(ws[i], st);
            if (rc != TM_OK) {
                tm_weights_destroy(ws[i]);
                ws[i] = nullptr;
                status[i] = rc;
            }
        } else {
            ws[i]->W = hW[i];
        }
    }
    timer.stop();
    TM_HIP(sync_stream(st));
    timer.finish();
    std::vector<tm_weights*> act;
    std::vector<u64> kk, ss;
    std::vector<int> idx;
    for (int i = 0; i < n_jobs; ++i) {
        if (!ws[i]) {
            std::memset(&out[i], 0, sizeof(tm_result));
            out[i].k = k[i];
            out[i].status = status[i];
            continue;
        }
        act.push_back(ws[i]);
        kk.push_back(k[i]);
        ss.push_back(seed[i]);
        idx.push_back(i);
    }
    int rc = TM_OK;
    if (!act.empty()) {
        std::vector<tm_result> r(act.size());
        rc = sample_batch_results(act.data(), reinterpret_cast<const uint64_t*>(kk.data()),
                                  reinterpret_cast<const uint64_t*>(ss.data()), (int)act.size(), st, r.data());
        for (size_t a = 0; a < act.size() && rc == TM_OK; ++a) out[idx[a]] = r[a];
    }
    for (tm_weights* w : ws) tm_weights_destroy(w);
    return rc;
}

// ---------------------------------------------------------------------------
// Batch plans: the 64-bit pipeline of a fixed job set recorded into a graph.
// ---------------------------------------------------------------------------
struct tm_batch_plan {
    int n = 0;
    std::vector<tm_graph*> g;
    std::vector<tm_motif> mo;
    std::vector<tm_tree> tr;
    std::vector<u64> k, seed;
    std::vector<tm_weights*> ws;
    int* flags = nullptr;  // per job: its 64-bit build overflowed
    u64* wdev = nullptr;   // per job: W (64-bit)
    CapturedPass* pass = nullptr;
    std::vector<std::pair<void*, hipStream_t>> kept;  // temporaries the graph reuses
    hipStream_t cs = nullptr;                         // the stream recorded on
    hipStream_t br[4] = {};                           // branches for the weight builds
    hipEvent_t ev[5] = {};                            // fork and joins
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static void plan_release(tm_batch_plan* p) {
    if (!p) return;
    if (p->cs) (void)sync_stream(p->cs);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    (void)hipDeviceSynchronize();
    if (p->pass) batch_capture_free(p->pass, p->cs);
    for (tm_weights* w : p->ws) tm_weights_destroy(w);
    for (auto& b : p->kept) (void)dev_free(b.first, b.second);
    (void)dev_free(p->flags, p->cs);
    (void)dev_free(p->wdev, p->cs);
    for (hipStream_t b : p->br)
        if (b) {
            (void)sync_stream(b);
            (void)hipStreamDestroy(b);
        }
    for (hipEvent_t e : p->ev)
        if (e) (void)hipEventDestroy(e);
    if (p->cs) {
        (void)sync_stream(p->cs);
        (void)hipStreamDestroy(p->cs);
    }
    delete p;
}

extern "C" int tm_batch_plan_create(tm_graph* const* g, const tm_motif* mo, const tm_tree* const* tr,
                                    const uint64_t* k, const uint64_t* seed, int n_jobs, void* stream,
                                    tm_batch_plan** out) {
    AllocScope scope_(g && n_jobs > 0 ? alloc_of(g[0]) : nullptr);
    (void)stream;
    if (!out || n_jobs < 1 || !g || !mo || !k || !seed) return tm_fail(TM_EINVAL, "batch_plan: bad arguments");
    std::unique_ptr<tm_batch_plan> P(new (std::nothrow) tm_batch_plan());
    if (!P) return tm_fail(TM_ENOMEM, "batch_plan: host allocation");
    P->n = n_jobs;
    std::vector<HostPlan> plans(n_jobs);
    for (int i = 0; i < n_jobs; ++i) {
        if (!g[i]) return tm_fail(TM_EINVAL, "batch_plan: job %d has no graph", i);
        TM_TRY(motif_check(&mo[i]));
        tm_tree t;
        if (tr && tr[i]) t = *tr[i];
        else TM_TRY(tm_default_tree(&mo[i], &t));
        TM_TRY(plan_build(&mo[i], &t, &plans[i]));
        if (g[i]->m > 0 && g[i]->T / mo[i].delta + 1 >= ((int64_t)1 << 31))
            return tm_fail(TM_ERANGE, "batch_plan: job %d has too many intervals", i);
        P->g.push_back(g[i]);
        P->mo.push_back(mo[i]);
        P->tr.push_back(t);
        P->k.push_back(k[i]);
        P->seed.push_back(seed[i]);
    }
    TM_HIP(hipStreamCreateWithFlags(&P->cs, hipStreamNonBlocking));
    tm_batch_plan* raw = P.release();
    auto fail = [&](int rc) {
        plan_release(raw);
        return rc;
    };
    for (hipStream_t& b : raw->br)
        if (hipStreamCreateWithFlags(&b, hipStreamNonBlocking) != hipSuccess)
            return fail(tm_fail(TM_EDEVICE, "batch_plan: cannot create a stream"));
    for (hipEvent_t& e : raw->ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return fail(tm_fail(TM_EDEVICE, "batch_plan: cannot create an event"));
    if (dev_alloc((void**)&raw->flags, n_jobs * sizeof(int), raw->cs) != hipSuccess ||
        dev_alloc((void**)&raw->wdev, n_jobs * sizeof(u64), raw->cs) != hipSuccess)
        return fail(tm_fail(TM_ENOMEM, "batch_plan: device allocation"));
    // weight builds go round-robin to the branches, largest graphs first
    constexpr int kBranches = 4;
    std::vector<int> order(n_jobs), branch(n_jobs, 0);
    for (int i = 0; i < n_jobs; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return raw->g[a]->m > raw->g[b]->m; });
    {
        int64_t load[kBranches] = {};
        for (int i : order) {
            int b = 0;
            for (int x = 1; x < kBranches; ++x)
                if (load[x] < load[b]) b = x;
            branch[i] = b;
            load[b] += raw->g[i]->m;
        }
    }
    raw->ws.assign(n_jobs, nullptr);
    for (int i = 0; i < n_jobs; ++i) {
        tm_weights* w = new (std::nothrow) tm_weights();
        if (!w) return fail(tm_fail(TM_ENOMEM, "batch_plan: host allocation"));
        w->g = raw->g[i];
        w->arena.stream = raw->br[branch[i]];
        w->plan = plans[i];
        raw->ws[i] = w;
    }
    // record: every 64-bit weight build, W of each job, the batched pass
    int rc = TM_OK;
    dev_defer_begin(&raw->kept);
    prof_suspend(true);
    hipError_t e = hipStreamBeginCapture(raw->cs, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) rc = tm_fail(TM_EDEVICE, "batch_plan: begin capture: %s", hipGetErrorString(e));
    if (rc == TM_OK) rc = fill_u32(raw->flags, n_jobs, 0u, raw->cs);
    if (rc == TM_OK) rc = fill_u32(raw->wdev, 2 * n_jobs, 0u, raw->cs);
    // fork: the branches start after the clears; join before the pass
    if (rc == TM_OK && hipEventRecord(raw->ev[0], raw->cs) != hipSuccess)
        rc = tm_fail(TM_EDEVICE, "batch_plan: fork");
    for (int b = 0; b < kBranches && rc == TM_OK; ++b)
        if (hipStreamWaitEvent(raw->br[b], raw->ev[0], 0) != hipSuccess) rc = tm_fail(TM_EDEVICE, "batch_plan: fork");
    for (int i : order) {
        if (rc != TM_OK) break;
        tm_weights* w = raw->ws[i];
        hipStream_t bs = raw->br[branch[i]];
        rc = weights_enqueue(w, bs, raw->flags + i);
        if (rc == TM_OK && w->q > 0 && w->cumW) {
            e = hipMemcpyAsync(raw->wdev + i, static_cast<const unsigned char*>(w->cumW) + w->q * 8, 8,
                               hipMemcpyDeviceToDevice, bs);
            if (e != hipSuccess) rc = tm_fail(TM_EDEVICE, "batch_plan: copy: %s", hipGetErrorString(e));
        }
    }
    for (int b = 0; b < kBranches && rc == TM_OK; ++b)
        if (hipEventRecord(raw->ev[1 + b], raw->br[b]) != hipSuccess ||
            hipStreamWaitEvent(raw->cs, raw->ev[1 + b], 0) != hipSuccess)
            rc = tm_fail(TM_EDEVICE, "batch_plan: join");
    if (rc == TM_OK) {
        std::vector<const int*> wf(n_jobs);
        for (int i = 0; i < n_jobs; ++i) wf[i] = raw->flags + i;
        rc = batch_capture_enqueue(raw->ws.data(), wf.data(), raw->k.data(), raw->seed.data(), n_jobs, raw->cs,
                                   batch_config_now(), &raw->pass);
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(raw->cs, &graph);
    prof_suspend(false);
    dev_defer_end();
    raw->graph = graph;
    if (rc == TM_OK && e != hipSuccess) rc = tm_fail(TM_EDEVICE, "batch_plan: end capture: %s", hipGetErrorString(e));
    if (rc == TM_OK) {
        e = hipGraphInstantiate(&raw->exec, raw->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = tm_fail(TM_EDEVICE, "batch_plan: instantiate: %s", hipGetErrorString(e));
    }
    if (rc != TM_OK) {
        (void)hipGetLastError();
        return fail(rc);
    }
    *out = raw;
    return TM_OK;
}

extern "C" int tm_batch_plan_run(tm_batch_plan* p, void* stream, tm_result* out) {
    if (!p || !out) return tm_fail(TM_EINVAL, "batch_plan_run: NULL argument");
    hipStream_t st = as_stream(stream);
    TM_HIP(hipGraphLaunch(p->exec, st));
    std::vector<int> hflags(p->n);
    std::vector<u64> hW(p->n);
    TM_HIP(read_back({{hflags.data(), p->flags, p->n * sizeof(int)}, {hW.data(), p->wdev, p->n * sizeof(u64)}}, st));
    std::vector<JobSums> sums(p->n);
    TM_TRY(batch_capture_read(p->pass, st, sums.data()));
    for (int i = 0; i < p->n; ++i) {
        tm_result& o = out[i];
        if (hflags[i]) {
            // 64 bits do not hold this job's weights: the 128-bit path, eagerly
            TM_TRY(tm_estimate(p->g[i], &p->mo[i], &p->tr[i], p->k[i], p->seed[i], stream, &o, nullptr));
            continue;
        }
        std::memset(&o, 0, sizeof o);
        o.k = p->k[i];
        o.q = p->ws[i]->q;
        o.W.lo = hW[i];
        o.W.hi = 0;
        if (hW[i] == 0) o.flags |= TM_F_W_ZERO;
        sums_to_result(sums[i], &o);
        if (o.status == TM_OK) finish_result(&o);
    }
    return TM_OK;
}

extern "C" void tm_batch_plan_destroy(tm_batch_plan* p) { plan_release(p); }

// ---------------------------------------------------------------------------
// Motif families (Sec. 4.3, Tab. "4-vertex-runtime"): several motifs from one
// sample stream of a shared spanning tree.
// ---------------------------------------------------------------------------
// The tree of w as a tree of motif mo: the same tree edges -- the same
// (source, destination) pairs, found once each and in the same relative
// order -- and the same delta; the plan must have w's slot structure.
static int family_plan(const tm_weights* w, const tm_motif* mo, HostPlan* out) {
    TM_TRY(motif_check(mo));
    const HostPlan& P0 = w->plan;
    if (P0.po) return tm_fail(TM_EINVAL, "family: the weight set's motif has a partial order");
    if (mo->k != P0.mo.k || mo->delta != P0.mo.delta)
        return tm_fail(TM_EINVAL, "family: motif differs in vertex count or delta");
    tm_tree t;
    std::memset(&t, 0, sizeof t);
    t.n_edges = P0.nt;
    int prev = -1;
    bool used[TM_MAX_L] = {false};
    for (int x = 0; x < P0.nt; ++x) {  // tree edges in increasing pi index
        const int s = P0.by_pi[x];
        const int e0 = P0.edge[s];
        int hit = -1;
        for (int p = 0; p < mo->l; ++p)
            if (!used[p] && mo->src[p] == P0.mo.src[e0] && mo->dst[p] == P0.mo.dst[e0]) {
                if (hit >= 0) return tm_fail(TM_EINVAL, "family: tree edge %d matches several edges", e0);
                hit = p;
            }
        if (hit < 0) return tm_fail(TM_EINVAL, "family: tree edge %d missing", e0);
        if (hit <= prev) return tm_fail(TM_EINVAL, "family: tree edges in another order");
        used[hit] = true;
        prev = hit;
        t.edge[x] = hit;
        if (e0 == P0.tree.center) t.center = hit;
    }
    TM_TRY(plan_build(mo, &t, out));
    const HostPlan& P = *out;
    if (P.po) return tm_fail(TM_EINVAL, "family: a member motif has a partial order");
    if (P.nt != P0.nt || P.H != P0.H) return tm_fail(TM_EINVAL, "family: tree shape differs");
    for (int s = 0; s < P.nt; ++s)
        if (P.parent[s] != P0.parent[s] || P.side[s] != P0.side[s] || P.alpha[s] != P0.alpha[s] ||
            P.beta[s] != P0.beta[s] || P.by_pi[s] != P0.by_pi[s] ||
            P.mo.src[P.edge[s]] != P0.mo.src[P0.edge[s]] || P.mo.dst[P.edge[s]] != P0.mo.dst[P0.edge[s]])
            return tm_fail(TM_EINVAL, "family: tree shape differs");
    return TM_OK;
}

extern "C" int tm_sample_family(tm_weights* w, const tm_motif* motifs, int n_motifs, uint64_t seed, uint64_t k,
                                void* stream, tm_result* out) {
    AllocScope scope_(w ? alloc_of(w->g) : nullptr);
    if (!w || !motifs || !out || n_motifs < 1 || n_motifs > 64)
        return tm_fail(TM_EINVAL, "sample_family: bad arguments");
    std::vector<HostPlan> plans(n_motifs);
    for (int f = 0; f < n_motifs; ++f) TM_TRY(family_plan(w, &motifs[f], &plans[f]));
    std::vector<JobSums> sums(n_motifs);
    JobSums shared;
    TM_TRY(family_run(w, plans.data(), n_motifs, seed, k, as_stream(stream), sums.data(), &shared));
    for (int f = 0; f < n_motifs; ++f) {
        tm_result& o = out[f];
        std::memset(&o, 0, sizeof o);
        o.k = k;
        o.q = w->q;
        o.W.lo = (u64)w->W;
        o.W.hi = (u64)(w->W >> 64);
        if (w->wide) o.flags |= TM_F_WIDE;
        if (w->W == 0) o.flags |= TM_F_W_ZERO;
        JobSums x = sums[f];
        x.n_valid = shared.n_valid;
        x.n_vertex = shared.n_vertex;
        x.n_delta = shared.n_delta;
        x.n_order = shared.n_order;
        sums_to_result(x, &o);
        if (o.status == TM_OK) finish_result(&o);
    }
    return TM_OK;
}

extern "C" int tm_list_instances(tm_weights* w, uint64_t seed, uint64_t j0, uint64_t count, void* stream,
                                 int32_t* eids, tm_sample_rec* recs) {
    AllocScope scope_(w ? alloc_of(w->g) : nullptr);
    if (!w || (count > 0 && !eids)) return tm_fail(TM_EINVAL, "list_instances: NULL argument");
    if (count > 0 && j0 + count < j0) return tm_fail(TM_EINVAL, "list_instances: id range wraps");
    if (w->plan.po) return tm_fail(TM_EINVAL, "list_instances: the motif has a partial order");
    return list_run(w, seed, j0, count, as_stream(stream), eids, recs);
}
