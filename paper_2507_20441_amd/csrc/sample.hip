// Sampling, validation, completion and reduction (Alg. 3 - Alg. 6).
//
// One lane per sample.  Draw 0 picks (interval, center edge) by inverse CDF
// over the pairs in (interval, eid) order: a search of the interval prefix
// W_i (staged in LDS when it fits), then of the center's prefix array inside
// the interval.  Each further tree edge, in pre-order, is drawn by inverse CDF
// over its candidate list: the window of the shared vertex's list minus the
// run of edges to the excluded vertex.  The excluded entries sit at known
// T-order positions (xref), so the number J of excluded entries before the
// answer is found by a search over the excluded run, and the answer by one
// more search of the window's prefix array at the target shifted by their
// weight.
//
// Each sample's state (matched eid, endpoints and time per tree slot, image
// per motif vertex) stays in registers: loops over tree slots are unrolled to
// the largest tree, and slot and vertex indices from the plan are uniform
// kernel arguments, resolved by selects rather than indexed memory.  Runs of
// three or more non-tree edges, or a leading and a trailing run coupled by
// delta, take a separate kernel variant with the general chain counter.
#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>
#include <type_traits>
#include <vector>

#include "tm_primitives.h"

namespace {

struct SampleArgs {
    DevGraph G;
    int64_t delta;
    int64_t ilen;  // interval unit (delta, or one interval over all times)
    int exclude;   // constraint 2: candidates exclude the parent's other endpoint
    int64_t q;
    int k;
    int nt;
    int esrc[kMaxSlots], edst[kMaxSlots];  // motif vertices of each slot's edge
    int parent[kMaxSlots], side[kMaxSlots], dir[kMaxSlots], beta[kMaxSlots], leaf[kMaxSlots];
    int new_vertex[kMaxSlots];
    int gv[kMaxSlots], ov[kMaxSlots];  // a child's shared motif vertex and its parent's other end
    int by_pi[kMaxSlots];
    int pi_pos[kMaxSlots];  // inverse of by_pi
    int same_window[kMaxSlots];
    const void* qt[kMaxSlots][2];
    const void* qn[kMaxSlots][2];
    int list_wide;  // the list tables hold 128-bit entries (else 64-bit, also under W = u128)
    const void* qtc[kMaxSlots][2];  // every 2^kCoarseBits-th entry of each qt table
    // kept child windows (see weights): parity par of the parent at list
    // position x is win[s][par][2 x] (the parities interleave), x the
    // parent's position in the T order of the list slot s attaches to
    // (side[s]); win_from[s]: the list the parent is drawn from, so that
    // when the two differ the parent's position is looked up (leid, tpos)
    const int4* win[kMaxSlots][2];
    int win_from[kMaxSlots];
    int has_win;
    int root_dir;  // the list whose T positions key the root (0: out-lists, 1: in-lists)
    const void* qc[2];
    const int32_t* ilo;
    const int32_t* ihi;
    const void* cumW;
    const RootGuide* guide;  // root pairs at 2^guide_bits + 1 evenly spaced draws (see weights)
    int guide_bits;
    const void* ioff;  // per interval: cum[i] - qc[lo_i]
    // captured passes: W read from the job's table, and the job skipped when
    // its 64-bit weight build overflowed (wflag set) or W = 0
    const void* Wdev;
    const int* wflag;
    int cum_in_lds;  // the q+1 interval prefix fits the block's LDS
    u64 W_lo, W_hi;
    int n_free;
    int free_src[TM_MAX_L], free_dst[TM_MAX_L];
    int n_runs;
    int run_first[TM_MAX_L], run_len[TM_MAX_L], run_prev[TM_MAX_L], run_next[TM_MAX_L];
    int general_runs;  // some run needs the general chain counter (3+ lists, or a
                       // leading and a trailing run coupled by delta), or the
                       // motif has a partial order
    // partial orders (po = 1): "strictly earlier" masks (see HostPlan)
    int po;
    uint16_t po_tpred[kMaxSlots];
    uint16_t po_f_tpred[kPoMaxFree], po_f_tsucc[kPoMaxFree], po_f_fpred[kPoMaxFree];
    u64 seed, j0, count;
    tm_sample_rec* recs;
    struct Partial* parts;
    int* ovf;
    const uint32_t* skey;  // root-sorted order: T-order position of the root * 2 + interval parity
    const uint32_t* sval;  // ... and the sample's offset in [0, count)
    uint32_t key_base;     // batched: skey of this job = key_base + its root key
};

// Per-lane running sums of a sampling pass.
struct LaneAcc {
    u128 acc2, acc2_sq;
    uint32_t n_valid, n_vertex, n_delta, n_order, n_nonzero;
    u64 flags, nb;
    bool ovf, bad;
};

struct Partial {
    u128 acc2, acc2_sq;
    u64 n_valid, n_vertex, n_delta, n_order, n_nonzero;
    u64 flags;  // bit 0: acc2 wrapped, bit 1: acc2_sq saturated
    u64 bytes;  // access-model bytes (counting pass only)
};

constexpr int kCumLdsBytes = 24 * 1024;

// Reads charged to one binary search over L entries: ceil(log2(L + 1)).
__device__ __forceinline__ u64 probes(int64_t L) { return L <= 0 ? 0 : (u64)(64 - __clzll((u64)L)); }

// Compile-time loop: f(integral_constant<I>) for I in [B, E).  Register
// arrays are only ever indexed by these constants, so they never become
// stack memory.
template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(static_cast<F&&>(f));
    }
}

template <int N, typename T>
__device__ __forceinline__ T pick(const T (&v)[N], int idx) {
    T r = v[0];
    sfor<1, N>([&](auto j) { r = (idx == decltype(j)::value) ? v[decltype(j)::value] : r; });
    return r;
}

template <int N, typename T>
__device__ __forceinline__ void put(T (&v)[N], int idx, T x) {
    sfor<0, N>([&](auto j) { v[decltype(j)::value] = (idx == decltype(j)::value) ? x : v[decltype(j)::value]; });
}

// ---------------------------------------------------------------------------
// Branchless searches.  Each step halves the candidate range; the final step
// settles the last element.  Several searches over the same range run in
// lockstep so that their loads are independent.
// ---------------------------------------------------------------------------
struct Bounds {
    int32_t p0, p1;  // T-order window [p0, p1)
    int32_t q0, q1;  // N-order excluded run [q0, q1)
    int32_t a, b;    // the vertex's list
};

// The four searches of window_bounds in lockstep over a T order of time
// type TT (wlo <= whi inside [0, T], which TT holds).
template <typename TT>
__device__ __forceinline__ void window_search(const TT* lt, const u64* nk, int32_t a, int32_t b, TT wlo, TT whi,
                                              u64 klo, u64 khi, Bounds& r) {
    int32_t b0 = a, b1 = a, b2 = a, b3 = a;
    int32_t n = b - a;
    while (n > 1) {
        const int32_t h = n >> 1;
        const TT x0 = lt[b0 + h], x1 = lt[b1 + h];
        const u64 x2 = nk[b2 + h], x3 = nk[b3 + h];
        b0 = x0 < wlo ? b0 + h : b0;
        b1 = x1 <= whi ? b1 + h : b1;
        b2 = x2 < klo ? b2 + h : b2;
        b3 = x3 <= khi ? b3 + h : b3;
        n -= h;
    }
    r.p0 = b0 + (lt[b0] < wlo ? 1 : 0);
    r.p1 = b1 + (lt[b1] <= whi ? 1 : 0);
    r.q0 = b2 + (nk[b2] < klo ? 1 : 0);
    r.q1 = b3 + (nk[b3] <= khi ? 1 : 0);
}

// The child window of Claim "matching-edges-set" in list dir of vertex g with
// time in [wlo, whi], and the run of edges whose far endpoint is o.
__device__ __forceinline__ Bounds window_bounds(const DevGraph& G, int dir, int32_t g, int32_t o,
                                                int64_t wlo, int64_t whi) {
    Bounds r;
    r.a = G.off[dir][g];
    r.b = G.off[dir][g + 1];
    if (wlo < 0) wlo = 0;
    if (whi > G.T) whi = G.T;
    if (wlo > whi || r.a == r.b) {
        r.p0 = r.p1 = r.q0 = r.q1 = r.a;
        return r;
    }
    const u64* nk = G.nkey[dir];
    const u64 base = (u64)o << G.bt;
    const u64 klo = base | (u64)wlo, khi = base | (u64)whi;
    if (G.lt32[dir])
        window_search<uint32_t>(G.lt32[dir], nk, r.a, r.b, (uint32_t)wlo, (uint32_t)whi, klo, khi, r);
    else
        window_search<int64_t>(G.lt[dir], nk, r.a, r.b, wlo, whi, klo, khi, r);
    return r;
}

// The multi-edge run El_{x,y} restricted to times [lo, hi].  It is a
// contiguous run both of x's out-list in (destination, time) order and of y's
// in-list in (source, time) order; [ra, rb) are its positions in list dir of
// those two (la, lb: the list searched).  ra is searched over the list; the
// run is short (the edges between one pair of vertices), so rb is found by
// galloping from ra (probes at doubling distances, then a search between the
// last two): a few probes instead of a second search of the whole list.
// np (counting variant): the probes made are added there.
__device__ __forceinline__ void el_run_dir(const DevGraph& G, int dir, int32_t x, int32_t y, int64_t lo, int64_t hi,
                                           int32_t la_in, int32_t lb_in, int32_t& ra, int32_t& rb, int32_t& la,
                                           int32_t& lb, u64* np = nullptr) {
    la = la_in;
    lb = lb_in;
    if (lo < 0) lo = 0;
    if (hi > G.T) hi = G.T;
    if (lo > hi || la == lb) {
        ra = rb = la;
        return;
    }
    const u64* nk = G.nkey[dir];
    const u64 base = (u64)(dir ? x : y) << G.bt;
    const u64 klo = base | (u64)lo, khi = base | (u64)hi;
    int32_t b0 = la;
    int32_t n = lb - la;
    while (n > 1) {
        const int32_t h = n >> 1;
        b0 = nk[b0 + h] < klo ? b0 + h : b0;
        n -= h;
        if (np) ++*np;
    }
    ra = b0 + (nk[b0] < klo ? 1 : 0);
    if (np) ++*np;
    // every key before ra is below klo <= khi: rb is the first position at
    // or after ra whose key exceeds khi; [g0, g1] holds it
    int32_t g0 = ra, g1 = lb, p = ra - 1;
    for (int32_t step = 1;; step <<= 1) {
        const int32_t q = p + step;
        if (q >= lb) break;
        if (np) ++*np;
        if (nk[q] > khi) {
            g1 = q;
            break;
        }
        g0 = q + 1;
        p = q;
    }
    while (g0 < g1) {
        const int32_t mid = g0 + ((g1 - g0) >> 1);
        if (np) ++*np;
        if (khi < nk[mid]) g1 = mid;
        else g0 = mid + 1;
    }
    rb = g0;
}

// El_{x,y} in the shorter of the two lists that hold it; returns that list's
// N-order keys (the run's times are their low bits).
__device__ __forceinline__ const u64* el_run(const DevGraph& G, int32_t x, int32_t y, int64_t lo, int64_t hi,
                                             int32_t& ra, int32_t& rb, int32_t& la, int32_t& lb, u64* np = nullptr) {
    const int32_t xa = G.off[0][x], xb = G.off[0][x + 1];
    const int32_t ya = G.off[1][y], yb = G.off[1][y + 1];
    const int dir = (yb - ya) < (xb - xa) ? 1 : 0;
    el_run_dir(G, dir, x, y, lo, hi, dir ? ya : xa, dir ? yb : xb, ra, rb, la, lb, np);
    return G.nkey[dir];
}

__device__ __forceinline__ u64 tmask_of(const DevGraph& G) {
    return G.bt >= 64 ? ~0ull : ((1ull << G.bt) - 1);
}

// ---------------------------------------------------------------------------
// Completion counting (Alg. 5).  A run of consecutive non-tree motif edges
// takes one edge from each of its multi-edge lists with strictly increasing
// times inside [lo, hi].  One list: its length.  Two lists: a two-pointer
// merge.  More lists, or a leading and a trailing run coupled by delta: the
// general counter below (a merge-sweep with one counter per list).
// ---------------------------------------------------------------------------
template <bool kCount>
__device__ __forceinline__ u128 run_count_short(const DevGraph& G, int32_t x0, int32_t y0, int32_t x1,
                                                int32_t y1, int len, int64_t lo, int64_t hi, u64& nb) {
    int32_t a0, b0, la0, lb0;
    u64 np = 0;  // probes of the run searches (counting variant)
    const u64* nk0 = el_run(G, x0, y0, lo, hi, a0, b0, la0, lb0, kCount ? &np : nullptr);
    if constexpr (kCount) nb += 16 + np * 8;
    if (len == 1) return (u128)(b0 - a0);
    int32_t a1, b1, la1, lb1;
    np = 0;
    const u64* nk1 = el_run(G, x1, y1, lo, hi, a1, b1, la1, lb1, kCount ? &np : nullptr);
    if constexpr (kCount) nb += 16 + np * 8 + (u64)(b0 - a0 + b1 - a1) * 8;
    // pairs (e, f), e in the first list, f in the second, t(e) < t(f)
    const u64 m = tmask_of(G);
    u128 total = 0;
    int32_t p = a0;
    for (int32_t f = a1; f < b1; ++f) {
        const u64 tf = nk1[f] & m;
        while (p < b0 && (nk0[p] & m) < tf) ++p;
        total += (u128)(p - a0);
    }
    return total;
}

struct V8 {
    int32_t v[TM_MAX_K];
};

// Chains through the lists of free edges first .. first+len-1 with times in
// [lo, hi]; merge-sweep in time order, later lists first on equal times.
template <bool kCount>
__device__ u128 chain_count_general(const DevGraph& G, const V8& img, const int* fs, const int* fd,
                                    int first, int len, int64_t lo, int64_t hi, bool* ovf, u64& nb) {
    if (len == 0) return 1;
    int32_t ra[TM_MAX_L], rb[TM_MAX_L];
    const u64* nks[TM_MAX_L];
    for (int j = 0; j < len; ++j) {
        int32_t la, lb;
        u64 np = 0;
        nks[j] = el_run(G, img.v[fs[first + j]], img.v[fd[first + j]], lo, hi, ra[j], rb[j], la, lb,
                        kCount ? &np : nullptr);
        if constexpr (kCount) nb += 16 + np * 8 + (u64)(rb[j] - ra[j]) * 8;
    }
    if (len == 1) return (u128)(rb[0] - ra[0]);
    const u64 m = tmask_of(G);
    u128 S[TM_MAX_L];
    for (int j = 0; j < len; ++j) S[j] = 0;
    while (true) {
        int best = -1;
        u64 tb = 0;
        for (int j = len - 1; j >= 0; --j) {
            if (ra[j] < rb[j]) {
                const u64 tj = nks[j][ra[j]] & m;
                if (best < 0 || tj < tb) {
                    tb = tj;
                    best = j;
                }
            }
        }
        if (best < 0) break;
        const u128 c = best == 0 ? (u128)1 : S[best - 1];
        if (!add_ok(S[best], c, &S[best])) *ovf = true;
        ++ra[best];
    }
    return S[len - 1];
}

// All runs of a valid sample when some run needs the general counter.
template <bool kCount>
__device__ __noinline__ u128 complete_general(const SampleArgs& a, const V8& img, int64_t tfirst,
                                              int64_t tlast, const int64_t* tprev, const int64_t* tnext,
                                              bool* ovf, u64* nbp) {
    const DevGraph& G = a.G;
    u64 nb = 0;
    u128 m_phi = 1;
    int lead = -1, trail = -1;
    for (int r = 0; r < a.n_runs && m_phi != 0; ++r) {
        if (a.run_prev[r] < 0) { lead = r; continue; }
        if (a.run_next[r] < 0) { trail = r; continue; }
        const u128 c = chain_count_general<kCount>(G, img, a.free_src, a.free_dst, a.run_first[r],
                                                   a.run_len[r], tprev[r] + 1, tnext[r] - 1, ovf, nb);
        if (!mul_ok(m_phi, c, &m_phi)) *ovf = true;
    }
    if (m_phi != 0 && lead >= 0 && trail < 0) {
        const u128 c = chain_count_general<kCount>(G, img, a.free_src, a.free_dst, a.run_first[lead],
                                                   a.run_len[lead], tlast - a.delta, tfirst - 1, ovf, nb);
        if (!mul_ok(m_phi, c, &m_phi)) *ovf = true;
    } else if (m_phi != 0 && trail >= 0 && lead < 0) {
        const u128 c = chain_count_general<kCount>(G, img, a.free_src, a.free_dst, a.run_first[trail],
                                                   a.run_len[trail], tlast + 1, tfirst + a.delta, ovf, nb);
        if (!mul_ok(m_phi, c, &m_phi)) *ovf = true;
    } else if (m_phi != 0 && trail >= 0 && lead >= 0) {
        // the first edge f of the leading chain fixes the end t(f) + delta of
        // the trailing chain
        int32_t fa, fb, la, lb;
        const int f0 = a.run_first[lead];
        u64 np = 0;
        const u64* nkf = el_run(G, img.v[a.free_src[f0]], img.v[a.free_dst[f0]], tlast - a.delta, tfirst - 1, fa,
                                fb, la, lb, kCount ? &np : nullptr);
        if constexpr (kCount) nb += 16 + np * 8 + (u64)(fb - fa) * 8;
        const u64 m = tmask_of(G);
        u128 sum = 0;
        for (int32_t x = fa; x < fb; ++x) {
            const int64_t tf = (int64_t)(nkf[x] & m);
            const u128 lc = chain_count_general<kCount>(G, img, a.free_src, a.free_dst, f0 + 1,
                                                        a.run_len[lead] - 1, tf + 1, tfirst - 1, ovf, nb);
            if (lc == 0) continue;
            const u128 tc = chain_count_general<kCount>(G, img, a.free_src, a.free_dst, a.run_first[trail],
                                                        a.run_len[trail], tlast + 1, tf + a.delta, ovf, nb);
            u128 prod;
            if (!mul_ok(lc, tc, &prod)) *ovf = true;
            if (!add_ok(sum, prod, &sum)) *ovf = true;
        }
        if (!mul_ok(m_phi, sum, &m_phi)) *ovf = true;
    }
    *nbp += nb;
    return m_phi;
}

// ---------------------------------------------------------------------------
// Completions under a partial order.  Each non-tree edge f takes an edge of
// its multi-edge list inside its bounds: after the tree edges that precede it
// and before those it precedes, and within delta of every tree time.  Among
// themselves the non-tree edges need their ordered pairs strictly in time
// order.  The count splits by the earliest time v of the whole match: all
// non-tree times in [t_min, t_min + delta] (the tree holds the earliest
// time), plus, for every candidate time v < t_min, the assignments inside
// [v, v + delta] with some non-tree edge at v.  Each part is one sweep over
// the candidates in time order (on equal times the later-listed edge first,
// so that an edge never follows one at its own time) with one count per set
// of assigned non-tree edges: an edge joins a set that holds everything it
// must follow.
// ---------------------------------------------------------------------------
struct PoRuns {
    int r;
    const u64* nk[kPoMaxFree];
    int32_t a[kPoMaxFree], b[kPoMaxFree];
};

// Assignments with every non-tree time in [lo, hi]; must: some non-tree edge
// at time lo exactly.
__device__ u128 po_sweep(const SampleArgs& a, const PoRuns& R, u64 tmask, int64_t lo, int64_t hi, bool must,
                         bool* ovf) {
    u128 dp[1 << kPoMaxFree];
    const int ns = 1 << R.r;
    for (int x = 0; x < ns; ++x) dp[x] = 0;
    dp[0] = 1;
    int32_t pos[kPoMaxFree];
    for (int f = 0; f < R.r; ++f) {
        int32_t x = R.a[f];
        while (x < R.b[f] && (int64_t)(R.nk[f][x] & tmask) < lo) ++x;
        pos[f] = x;
    }
    bool dropped = !must;
    while (true) {
        int best = -1;
        int64_t tb = 0;
        for (int f = R.r - 1; f >= 0; --f) {
            if (pos[f] >= R.b[f]) continue;
            const int64_t tf = (int64_t)(R.nk[f][pos[f]] & tmask);
            if (tf > hi) continue;
            if (best < 0 || tf < tb) {
                best = f;
                tb = tf;
            }
        }
        if (best < 0) break;
        if (!dropped && tb > lo) {
            dp[0] = 0;  // the sets with nothing at lo end here
            dropped = true;
        }
        const uint32_t need = a.po_f_fpred[best];
        const int bit = 1 << best;
        for (int S = 0; S < ns; ++S) {
            if ((S & bit) || (need & ~(uint32_t)S) || dp[S] == 0) continue;
            if (!add_ok(dp[S | bit], dp[S], &dp[S | bit])) *ovf = true;
        }
        ++pos[best];
    }
    return dp[ns - 1];
}

template <bool kCount>
__device__ __noinline__ u128 complete_po(const SampleArgs& a, const V8& img, const int64_t* te, bool* ovf, u64* nbp) {
    const DevGraph& G = a.G;
    if (a.n_free == 0) return 1;
    int64_t tlo = te[0], thi = te[0];
    for (int s = 1; s < a.nt; ++s) {
        tlo = te[s] < tlo ? te[s] : tlo;
        thi = te[s] > thi ? te[s] : thi;
    }
    PoRuns R;
    R.r = a.n_free;
    u64 nb = 0;
    for (int f = 0; f < R.r; ++f) {
        int64_t lo = thi - a.delta, hi = tlo + a.delta;
        for (int s = 0; s < a.nt; ++s) {
            if ((a.po_f_tpred[f] >> s) & 1u) lo = te[s] + 1 > lo ? te[s] + 1 : lo;
            if ((a.po_f_tsucc[f] >> s) & 1u) hi = te[s] - 1 < hi ? te[s] - 1 : hi;
        }
        if (lo > hi) {
            *nbp += nb;
            return 0;
        }
        int32_t la, lb;
        u64 np = 0;
        R.nk[f] = el_run(G, img.v[a.free_src[f]], img.v[a.free_dst[f]], lo, hi, R.a[f], R.b[f], la, lb,
                         kCount ? &np : nullptr);
        if constexpr (kCount) nb += 16 + np * 8 + (u64)(R.b[f] - R.a[f]) * 8;
        if (R.a[f] >= R.b[f]) {
            *nbp += nb;
            return 0;
        }
    }
    const u64 tmask = tmask_of(G);
    u128 total = po_sweep(a, R, tmask, tlo, tlo + a.delta, false, ovf);
    // anchors: the distinct candidate times below t_min, in increasing order
    int32_t cur[kPoMaxFree];
    for (int f = 0; f < R.r; ++f) cur[f] = R.a[f];
    while (true) {
        int64_t v = -1;
        for (int f = 0; f < R.r; ++f) {
            if (cur[f] >= R.b[f]) continue;
            const int64_t tf = (int64_t)(R.nk[f][cur[f]] & tmask);
            if (v < 0 || tf < v) v = tf;
        }
        if (v < 0 || v >= tlo) break;
        const u128 c = po_sweep(a, R, tmask, v, v + a.delta, true, ovf);
        if (!add_ok(total, c, &total)) *ovf = true;
        for (int f = 0; f < R.r; ++f)
            while (cur[f] < R.b[f] && (int64_t)(R.nk[f][cur[f]] & tmask) == v) ++cur[f];
        if constexpr (kCount) {
            for (int f = 0; f < R.r; ++f) nb += (u64)(R.b[f] - R.a[f]) * 8;
        }
    }
    *nbp += nb;
    return total;
}

// ---------------------------------------------------------------------------
// Wave and block reduction of the per-lane partial sums.
// ---------------------------------------------------------------------------
__device__ __forceinline__ u128 shfl_xor_u128(u128 v, int m) {
    const u64 lo = __shfl_xor((u64)v, m, 64), hi = __shfl_xor((u64)(v >> 64), m, 64);
    return ((u128)hi << 64) | lo;
}

__device__ __forceinline__ void combine(Partial& x, const Partial& y) {
    if (!add_ok(x.acc2, y.acc2, &x.acc2)) x.flags |= 1;
    if (!add_ok(x.acc2_sq, y.acc2_sq, &x.acc2_sq)) {
        x.acc2_sq = ~(u128)0;
        x.flags |= 2;
    }
    x.n_valid += y.n_valid;
    x.n_vertex += y.n_vertex;
    x.n_delta += y.n_delta;
    x.n_order += y.n_order;
    x.n_nonzero += y.n_nonzero;
    x.flags |= y.flags;
    x.bytes += y.bytes;
}

__device__ __forceinline__ void block_reduce_write(Partial acc, Partial* out) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        Partial y;
        y.acc2 = shfl_xor_u128(acc.acc2, m);
        y.acc2_sq = shfl_xor_u128(acc.acc2_sq, m);
        y.n_valid = __shfl_xor(acc.n_valid, m, 64);
        y.n_vertex = __shfl_xor(acc.n_vertex, m, 64);
        y.n_delta = __shfl_xor(acc.n_delta, m, 64);
        y.n_order = __shfl_xor(acc.n_order, m, 64);
        y.n_nonzero = __shfl_xor(acc.n_nonzero, m, 64);
        y.flags = __shfl_xor(acc.flags, m, 64);
        y.bytes = __shfl_xor(acc.bytes, m, 64);
        combine(acc, y);
    }
    __shared__ Partial red[kWaves];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        Partial s = red[0];
        for (int w = 1; w < kWaves; ++w) combine(s, red[w]);
        *out = s;
    }
}

// ---------------------------------------------------------------------------
// The sampling kernel.
// ---------------------------------------------------------------------------
// Draw 0 of sample a.j0 + r: the interval, then the center edge; returned as
// the root key (T-order position of the root * 2 + interval parity).
// Inconsistent tables give a harmless key and set bad.
// The job's W: read from its table when the host has not read it yet (Wdev),
// else from the arguments.
template <typename W>
__device__ __forceinline__ W job_W(const SampleArgs& a) {
    return a.Wdev ? *static_cast<const W*>(a.Wdev) : (W)(((u128)a.W_hi << 64) | a.W_lo);
}

// A job whose 64-bit weight build overflowed (wflag set) or whose W is 0
// draws nothing (its tables are not to be searched).
template <typename W>
__device__ __forceinline__ bool job_skipped(const SampleArgs& a, W Wtot) {
    return (a.wflag && *a.wflag != 0) || Wtot == 0;
}

template <typename W>
__device__ __forceinline__ bool draw_root_from(const SampleArgs& a, const W* cum, W Wtot, const X128& X,
                                               const RootGuide& g0, const RootGuide& g1, int32_t& i,
                                               int32_t& e0, u64* nb = nullptr, uint32_t* key = nullptr) {
    int32_t i0 = 0, i1 = (int32_t)a.q - 1, ea = -1, eb = 0x7fffffff;
    if (a.guide) {
        // the guide bucket of X bounds the pair between two guide entries;
        // equal ends leave one pair (the pair is monotone in X)
        i0 = (int32_t)(g0.pair >> 32);
        ea = (int32_t)(uint32_t)g0.pair;
        i1 = (int32_t)(g1.pair >> 32);
        eb = (int32_t)(uint32_t)g1.pair;
        if (g0.pair == g1.pair && i0 >= 0 && i0 < a.q) {
            i = i0;
            e0 = ea;
            if (key) *key = (uint32_t)g0.key;
            if (nb) *nb += 2 * sizeof(RootGuide);
            return true;
        }
    }
    const W r0 = scale(X, Wtot);
    int32_t span = 0;
    const bool ok = root_pair<W>(cum, a.qc, a.ilo, a.ihi, a.q, r0, i0, i1, ea, eb, i, e0, &span,
                                 static_cast<const W*>(a.ioff));
    if (nb) {
        if (a.ioff && i0 == i1) *nb += 2 * sizeof(RootGuide) + (1 + probes(span)) * sizeof(W);
        else *nb += (a.guide ? 2 * sizeof(RootGuide) : 0) + (probes(i1 - i0 + 1) + 2 + probes(span)) * sizeof(W) + 8;
    }
    return ok;
}

// The two guide entries around draw X (none without a guide).
__device__ __forceinline__ void guide_pair(const SampleArgs& a, const X128& X, RootGuide& g0, RootGuide& g1) {
    if (a.guide) {
        const u64 b = X.hi >> (64 - a.guide_bits);
        g0 = a.guide[b];
        g1 = a.guide[b + 1];
    } else {
        g0.pair = g1.pair = g0.key = g1.key = 0;
    }
}

template <typename W>
__device__ __forceinline__ bool draw_root(const SampleArgs& a, const W* cum, W Wtot, u64 j, int32_t& i,
                                          int32_t& e0, u64* nb = nullptr, uint32_t* key = nullptr) {
    const X128 X = draw_block(a.seed, j, 0);
    RootGuide g0, g1;
    guide_pair(a, X, g0, g1);
    return draw_root_from<W>(a, cum, Wtot, X, g0, g1, i, e0, nb, key);
}

// Draw 0 of sample a.j0 + r: the interval, then the center edge; returned as
// the root key (T-order position of the root * 2 + interval parity).
// Inconsistent tables give a harmless key and set bad.
template <typename W>
__device__ __forceinline__ uint32_t root_key(const SampleArgs& a, const W* cum, W Wtot, const X128& X,
                                             const RootGuide& g0, const RootGuide& g1, bool& bad) {
    int32_t i, e0;
    uint32_t key = ~0u;  // set by a one-pair guide bucket
    if (!draw_root_from<W>(a, cum, Wtot, X, g0, g1, i, e0, nullptr, &key)) {
        bad = true;
        return 0u;
    }
    return key != ~0u ? key : (uint32_t)a.G.tpos[a.root_dir][e0] * 2u + (uint32_t)(i & 1);
}

// Draw 0 of each sample (interval, then center edge), written as a sort key:
// the root's position in the T order of the root list (out-lists, or
// in-lists when every child of the center attaches at its destination:
// grouping samples by the vertex their first children share, then time) and
// the interval's parity.  The sort that follows changes only the order in
// which samples are processed.
template <typename W>
__global__ void __launch_bounds__(kBlock) root_kernel(SampleArgs a, uint32_t* keys, uint32_t* vals) {
    extern __shared__ unsigned char lds_raw[];
    const W Wtot = job_W<W>(a);
    const u64 count = job_skipped<W>(a, Wtot) ? 0 : a.count;
    const W* cumG = static_cast<const W*>(a.cumW);
    const int32_t ncum = (int32_t)a.q + 1;
    W* cumL = reinterpret_cast<W*>(lds_raw);
    if (a.cum_in_lds) {
        for (int32_t x = threadIdx.x; x < ncum; x += kBlock) cumL[x] = cumG[x];
        __syncthreads();
    }
    const W* cum = a.cum_in_lds ? cumL : cumG;
    bool bad = false;
    const u64 stride = (u64)gridDim.x * kBlock;
    (void)vals;  // the sort makes the sample offsets (0 .. count-1) itself
    // two draws per lane and step, both guide reads issued before either is
    // used: the random guide reads are the kernel's latency
    for (u64 r = (u64)blockIdx.x * kBlock + threadIdx.x; r < count; r += 2 * stride) {
        const u64 r1 = r + stride;
        const bool two = r1 < count;
        const X128 X0 = draw_block(a.seed, a.j0 + r, 0);
        const X128 X1 = draw_block(a.seed, a.j0 + (two ? r1 : r), 0);
        RootGuide g00, g01, g10, g11;
        guide_pair(a, X0, g00, g01);
        guide_pair(a, X1, g10, g11);
        keys[r] = root_key<W>(a, cum, Wtot, X0, g00, g01, bad);
        if (two) keys[r1] = root_key<W>(a, cum, Wtot, X1, g10, g11, bad);
    }
    if (bad) atomicOr(a.ovf, 2);
}

// Samples at positions x = x0, x0 + stride, ... < xend: sample offsets in
// [0, count), or, in root-sorted order, positions of the sorted arrays.
// M_phi of a valid tree image (Alg. 5): the completions over the non-tree
// edges of a's motif.  img: the graph vertex of every motif vertex; te: the
// time of every tree slot.
// ga: the same arguments where the no-inline routines read them (an LDS copy
// in the single-job kernel, so that the kernel's arguments are never copied
// to scratch for them).
template <bool kCount, bool kGeneral, int NT, int K>
__device__ __forceinline__ u128 completions(const SampleArgs& a, const SampleArgs& ga, const int32_t (&img)[K],
                                            const int64_t (&te)[NT], bool& ovf, u64& nb) {
    const DevGraph& G = a.G;
    u128 m_phi = 0;
    const int64_t tfirst = pick(te, a.by_pi[0]), tlast = pick(te, a.by_pi[a.nt - 1]);
    if constexpr (kGeneral) {
        V8 iv;
        sfor<0, TM_MAX_K>([&](auto x) {
            constexpr int xi = decltype(x)::value;
            iv.v[xi] = xi < K ? img[xi < K ? xi : 0] : -1 - xi;
        });
        if (a.po) {
            int64_t tt[kMaxSlots];
            sfor<0, kMaxSlots>([&](auto sc) {
                constexpr int si = decltype(sc)::value;
                tt[si] = si < NT ? te[si < NT ? si : 0] : 0;
            });
            m_phi = complete_po<kCount>(ga, iv, tt, &ovf, &nb);
        } else {
            int64_t tp[TM_MAX_L], tn[TM_MAX_L];
            for (int r2 = 0; r2 < a.n_runs; ++r2) {
                tp[r2] = a.run_prev[r2] >= 0 ? pick(te, a.run_prev[r2]) : 0;
                tn[r2] = a.run_next[r2] >= 0 ? pick(te, a.run_next[r2]) : 0;
            }
            m_phi = complete_general<kCount>(ga, iv, tfirst, tlast, tp, tn, &ovf, &nb);
        }
    } else {
        m_phi = 1;
        for (int r2 = 0; r2 < a.n_runs && m_phi != 0; ++r2) {
            const int pv = a.run_prev[r2], nx = a.run_next[r2];
            const int f0 = a.run_first[r2], len = a.run_len[r2];
            int64_t lo_t, hi_t;
            if (pv >= 0 && nx >= 0) {
                lo_t = pick(te, pv) + 1;
                hi_t = pick(te, nx) - 1;
            } else if (nx >= 0) {  // leading run only
                lo_t = tlast - a.delta;
                hi_t = tfirst - 1;
            } else {  // trailing run only
                lo_t = tlast + 1;
                hi_t = tfirst + a.delta;
            }
            const int32_t x0 = pick(img, a.free_src[f0]), y0 = pick(img, a.free_dst[f0]);
            const int32_t x1 = len > 1 ? pick(img, a.free_src[f0 + 1]) : 0;
            const int32_t y1 = len > 1 ? pick(img, a.free_dst[f0 + 1]) : 0;
            const u128 c = run_count_short<kCount>(G, x0, y0, x1, y1, len, lo_t, hi_t, nb);
            if (!mul_ok(m_phi, c, &m_phi)) ovf = true;
        }
    }
    return m_phi;
}

// kWin (root-sorted only): each child's window is read from the kept table
// at its parent's list position instead of searched for.
// kSmall: trees of at most four edges and motifs of at most five vertices,
// so that fewer register slots are live (more waves per SIMD).
// kNarrow (W = u128 only): a widened set whose list tables stayed 64-bit;
// its child masses fit 64 bits, so the child picks run in 64-bit arithmetic
// (the same draws: floor(X n / 2^128) does not depend on the width n is
// held in), and only the root draw is 128-bit.
template <typename W, bool kCount, bool kGeneral, bool kSorted, bool kWin = false, bool kSmall = false,
          bool kNarrow = false>
__device__ __forceinline__ void sample_positions(const SampleArgs& a, const SampleArgs& ga, const W* cum, u64 x0,
                                                 u64 xend, u64 stride, LaneAcc& L) {
    static_assert(kSorted || !kWin, "windows are read by list position");
    static_assert(!kNarrow || sizeof(W) == 16, "only a 128-bit set has narrower list tables");
    using WC = typename std::conditional<kNarrow, u64, W>::type;  // child-pick arithmetic
    constexpr int NT = kSmall ? 4 : kMaxSlots - 1;  // register slots; a.nt of them are used
    constexpr int K = kSmall ? 5 : TM_MAX_K;         // motif vertices held
    const DevGraph& G = a.G;
    u128 acc2 = L.acc2, acc2_sq = L.acc2_sq;
    uint32_t n_valid = L.n_valid, n_vertex = L.n_vertex, n_delta = L.n_delta, n_order = L.n_order,
             n_nonzero = L.n_nonzero;
    u64 flags = L.flags, nb = L.nb;
    bool ovf = L.ovf, bad = L.bad;
    for (u64 x = x0; x < xend; x += stride) {
        int64_t te[NT];
        int32_t posv[NT];  // kWin: each slot's position in the list it was drawn from
        int32_t img[K];
        sfor<0, K>([&](auto xx) { img[decltype(xx)::value] = -1 - decltype(xx)::value; });
        u64 r;
        int32_t i, e0, u0, v0;
        if constexpr (kSorted) {
            // the root was drawn by root_kernel; lanes follow the sorted order
            const uint32_t key = a.skey[x] - a.key_base;
            r = a.sval[x];
            const int32_t pos = (int32_t)(key >> 1);
            if constexpr (kWin) posv[0] = pos;
            const int rd = a.root_dir;
            e0 = G.leid[rd][pos];
            int32_t nbr0;
            list_entry(G.lnt[rd], G.lnbr[rd], G.lt[rd], pos, nbr0, te[0]);
            const int32_t own0 = G.lown[rd] ? G.lown[rd][pos] : (rd ? G.dst[e0] : G.src[e0]);
            u0 = rd ? nbr0 : own0;
            v0 = rd ? own0 : nbr0;
            const int64_t blk = te[0] / a.ilen;
            i = (int32_t)(((blk & 1) == (int64_t)(key & 1)) ? blk : blk - 1);
            if constexpr (kCount) nb += 8 + 12 + (G.lt32[0] ? 4 : 8);
        } else {
            // draw 0: interval, then center edge
            r = x;
            if (!draw_root<W>(a, cum, job_W<W>(a), a.j0 + r, i, e0, kCount ? &nb : nullptr)) {
                bad = true;
                break;
            }
            if constexpr (kCount) nb += 16;
            te[0] = G.t[e0];
            u0 = G.src[e0];
            v0 = G.dst[e0];
        }
        const u64 j = a.j0 + r;
        const int par = i & 1;
        put(img, a.esrc[0], u0);
        put(img, a.edst[0], v0);
        // matched eids go straight to the record, at the slot's rank in pi
        if (a.recs) a.recs[r].eid[a.pi_pos[0]] = e0;
        const int64_t ilo_t = (int64_t)i * a.ilen, ihi_t = ((int64_t)i + 2) * a.ilen - 1;
        Bounds last;  // the previous child's window, reused by a leaf sibling with the same one
        last.p0 = last.p1 = last.q0 = last.q1 = last.a = last.b = 0;
        // draws 1..nt-1: children in pre-order.  A runtime loop: the slot's
        // plan entries are read inside it rather than held for every slot.
#pragma unroll 1
        for (int s = 1; s < a.nt; ++s) {
            const int64_t pt = pick(te, a.parent[s]);
            const int32_t g = pick(img, a.gv[s]);
            const int32_t o = pick(img, a.ov[s]);
            // [t - delta, t] before the parent, [t, t + delta] after it,
            // [t - delta, t + delta] when a partial order leaves them unordered
            int64_t wlo = a.beta[s] > 0 ? pt : pt - a.delta;
            int64_t whi = a.beta[s] < 0 ? pt : pt + a.delta;
            wlo = wlo > ilo_t ? wlo : ilo_t;
            whi = whi < ihi_t ? whi : ihi_t;
            const int d = a.dir[s];
            Bounds w;
            if (a.same_window[s]) {
                w = last;
            } else if constexpr (kWin) {
                int32_t wx = pick(posv, a.parent[s]);
                if (a.win_from[s] != a.side[s]) {
                    // the parent was drawn from its other list: its position
                    // in the list the windows follow, through its eid
                    const int32_t pe = G.leid[a.win_from[s]][wx];
                    wx = G.tpos[a.side[s]][pe];
                    if constexpr (kCount) nb += 8;
                }
                const int4 b = a.win[s][par][2 * (int64_t)wx];
                w.p0 = b.x;
                w.p1 = b.y;
                w.q0 = b.z;
                w.q1 = b.w;
                w.a = w.b = 0;
            } else {
                w = window_bounds(G, d, g, o, wlo, whi);
            }
            if (!a.exclude) w.q1 = w.q0;  // constraint 2 off: nothing excluded
            last = w;
            const bool leaf = a.leaf[s] != 0;
            const ListTab<WC> qt{a.qt[s][par], !kNarrow && a.list_wide != 0, a.qtc[s][par], kCoarseBits};
            const ListTab<WC> qn{a.qn[s][par], !kNarrow && a.list_wide != 0};
            WC bt0 = 0, bn0 = 0, mass;
            if (leaf) {
                mass = (WC)((w.p1 - w.p0) - (w.q1 - w.q0));
            } else {
                bt0 = qt[w.p0];
                bn0 = qn[w.q0];
                mass = (qt[w.p1] - bt0) - (qn[w.q1] - bn0);
            }
            // a child of a positive-weight match always has positive mass
            if (mass == 0 || w.p1 <= w.p0) { bad = true; break; }
            const WC rr = scale(draw_block(a.seed, j, (uint32_t)s), mass);
            // J: excluded entries whose preceding candidate mass is <= rr
            const int32_t* xref = G.nxref[d];
            int32_t jb = w.q0, jn = w.q1 - w.q0;
            if (jn > 0) {
                while (jn > 1) {
                    const int32_t h = jn >> 1;
                    const int32_t mid = jb + h;
                    const int32_t xp = xref[mid];
                    const WC F = leaf ? (WC)((xp - w.p0) - (mid - w.q0)) : (qt[xp] - bt0) - (qn[mid] - bn0);
                    jb = F <= rr ? mid : jb;
                    jn -= h;
                }
                const int32_t xp = xref[jb];
                const WC F = leaf ? (WC)((xp - w.p0) - (jb - w.q0)) : (qt[xp] - bt0) - (qn[jb] - bn0);
                jb += F <= rr ? 1 : 0;
            }
            const int32_t J = jb - w.q0;
            int32_t pos;
            if (leaf) {
                pos = w.p0 + (int32_t)rr + J;
            } else {
                const WC tgt = bt0 + rr + (qn[w.q0 + J] - bn0);
                pos = qt.upper_bound_coarse(w.p0 + 1, w.p1 + 1, tgt) - 1;
            }
            pos = pos < w.p0 ? w.p0 : (pos >= w.p1 ? w.p1 - 1 : pos);
            if constexpr (kCount) {
                if (!a.same_window[s]) {
                    if constexpr (kWin) nb += sizeof(int4);
                    else
                        nb += 8 + (probes(w.b - w.a) + probes(w.b - w.p0)) * (G.lt32[0] ? 4 : 8) +
                              (probes(w.b - w.a) + probes(w.b - w.q0)) * 8;
                }
                nb += probes(w.q1 - w.q0) * (4 + (leaf ? 0 : 2 * qt.bytes()));
                if (!leaf) nb += (5 + probes(w.p1 - w.p0)) * qt.bytes();  // charged as the plain search
                nb += 8 + (G.lt32[0] ? 4 : 8);
            }
            int32_t nbv;
            int64_t tv;
            list_entry(G.lnt[d], G.lnbr[d], G.lt[d], pos, nbv, tv);
            put(te, s, tv);
            if constexpr (kWin) put(posv, s, pos);
            if (a.recs) a.recs[r].eid[a.pi_pos[s]] = G.leid[d][pos];
            put(img, a.new_vertex[s], nbv);
        }
        if (bad) break;
        // Alg. 4: vertex map 1-1, then delta range, then edge order
        uint32_t status = 0;
        sfor<0, K>([&](auto xc) {
            constexpr int x = decltype(xc)::value;
            sfor<x + 1, K>([&](auto yc) {
                constexpr int y = decltype(yc)::value;
                if (y < a.k && img[x] == img[y]) status = 1;
            });
        });
        int64_t tmin = te[0], tmax = te[0];
        sfor<1, NT>([&](auto sc) {
            constexpr int s = decltype(sc)::value;
            if (s < a.nt) {
                tmin = te[s] < tmin ? te[s] : tmin;
                tmax = te[s] > tmax ? te[s] : tmax;
            }
        });
        if (status == 0 && tmax - tmin > a.delta) status = 2;
        if constexpr (kGeneral) {
            if (status == 0 && a.po) {
                // a partial order: every ordered pair of tree edges in order
                sfor<0, NT>([&](auto xc) {
                    constexpr int x = decltype(xc)::value;
                    sfor<0, NT>([&](auto yc) {
                        constexpr int y = decltype(yc)::value;
                        if (x < a.nt && y < a.nt && ((a.po_tpred[x] >> y) & 1u) && !(te[y] < te[x])) status = 3;
                    });
                });
            }
        }
        if (status == 0 && !(kGeneral && a.po)) {
            sfor<1, NT>([&](auto xc) {
                constexpr int x = decltype(xc)::value;
                if (x < a.nt && !(pick(te, a.by_pi[x - 1]) < pick(te, a.by_pi[x]))) status = 3;
            });
        }
        uint32_t n_phi = 0;
        u128 m_phi = 0;
        if (status == 0) {
            // N_phi: intervals holding every tree edge (I_b always; I_{b-1}
            // when the last time is still below (b+1) L)
            const int64_t b = tmin / a.ilen;
            n_phi = (b < a.q ? 1u : 0u) + ((b >= 1 && tmax < (b + 1) * a.ilen) ? 1u : 0u);
            // Alg. 5: completions over the non-tree edges
            m_phi = completions<kCount, kGeneral, NT, K>(a, ga, img, te, ovf, nb);
            ++n_valid;
            if (m_phi != 0) ++n_nonzero;
            u128 term;
            if (!mul_ok(m_phi, (u128)(2 / n_phi), &term)) ovf = true;
            if (!add_ok(acc2, term, &acc2)) flags |= 1;
            u128 sq;
            if (!mul_ok(term, term, &sq) || !add_ok(acc2_sq, sq, &acc2_sq)) {
                acc2_sq = ~(u128)0;
                flags |= 2;
            }
        } else if (status == 1) {
            ++n_vertex;
        } else if (status == 2) {
            ++n_delta;
        } else {
            ++n_order;
        }
        if (a.recs) {
            tm_sample_rec& out = a.recs[r];
            out.interval = (uint32_t)i;
            out.status = status;
            out.n_phi = n_phi;
            out.pad = 0;
            sfor<1, 8>([&](auto xc) {
                constexpr int x = decltype(xc)::value;
                if (x >= a.nt) out.eid[x] = -1;
            });
            out.m_phi.lo = (u64)m_phi;
            out.m_phi.hi = (u64)(m_phi >> 64);
        }
    }
    L.acc2 = acc2;
    L.acc2_sq = acc2_sq;
    L.n_valid = n_valid;
    L.n_vertex = n_vertex;
    L.n_delta = n_delta;
    L.n_order = n_order;
    L.n_nonzero = n_nonzero;
    L.flags = flags;
    L.nb = nb;
    L.ovf = ovf;
    L.bad = bad;
}

__device__ __forceinline__ LaneAcc lane_zero() {
    LaneAcc L;
    L.acc2 = 0;
    L.acc2_sq = 0;
    L.n_valid = L.n_vertex = L.n_delta = L.n_order = L.n_nonzero = 0;
    L.flags = L.nb = 0;
    L.ovf = L.bad = false;
    return L;
}

// Block-wide sum of the lanes' partials into *out; flags into *ovf.
__device__ __forceinline__ void lanes_reduce(const LaneAcc& L, Partial* out, int* ovf) {
    Partial acc;
    acc.acc2 = L.acc2;
    acc.acc2_sq = L.acc2_sq;
    acc.n_valid = L.n_valid;
    acc.n_vertex = L.n_vertex;
    acc.n_delta = L.n_delta;
    acc.n_order = L.n_order;
    acc.n_nonzero = L.n_nonzero;
    acc.flags = L.flags;
    acc.bytes = L.nb;
    block_reduce_write(acc, out);
    if (L.ovf) atomicOr(ovf, 1);
    if (L.bad) atomicOr(ovf, 2);
}

template <typename W, bool kCount, bool kGeneral, bool kSorted, bool kWin, bool kSmall = false, bool kNarrow = false>
__global__ void __launch_bounds__(kBlock) sample_kernel(SampleArgs a) {
    extern __shared__ unsigned char lds_raw[];
    const W* cumG = static_cast<const W*>(a.cumW);
    const int32_t ncum = (int32_t)a.q + 1;
    W* cumL = reinterpret_cast<W*>(lds_raw);
    if (!kSorted && a.cum_in_lds) {
        for (int32_t x = threadIdx.x; x < ncum; x += kBlock) cumL[x] = cumG[x];
        __syncthreads();
    }
    const W* cum = a.cum_in_lds ? cumL : cumG;
    LaneAcc L = lane_zero();
    if (job_skipped<W>(a, job_W<W>(a))) {
        lanes_reduce(L, &a.parts[blockIdx.x], a.ovf);  // nothing drawn
        return;
    }
    if constexpr (kGeneral) {
        // the general variants' no-inline completion routines read the
        // arguments from an LDS copy (a reference to the kernel's own would
        // make it copy them to scratch in every lane)
        __shared__ SampleArgs s_args;
        if (threadIdx.x == 0) s_args = a;
        __syncthreads();
        sample_positions<W, kCount, kGeneral, kSorted, kWin, kSmall, kNarrow>(
            a, s_args, cum, (u64)blockIdx.x * kBlock + threadIdx.x, a.count, (u64)gridDim.x * kBlock, L);
    } else {
        sample_positions<W, kCount, kGeneral, kSorted, kWin, kSmall, kNarrow>(
            a, a, cum, (u64)blockIdx.x * kBlock + threadIdx.x, a.count, (u64)gridDim.x * kBlock, L);
    }
    lanes_reduce(L, &a.parts[blockIdx.x], a.ovf);
}

// Sum of the block partials (integers: the order does not matter).
__global__ void __launch_bounds__(kBlock) reduce_kernel(const Partial* parts, int n, Partial* out) {
    Partial acc;
    acc.acc2 = 0;
    acc.acc2_sq = 0;
    acc.n_valid = acc.n_vertex = acc.n_delta = acc.n_order = acc.n_nonzero = 0;
    acc.flags = 0;
    acc.bytes = 0;
    for (int b = threadIdx.x; b < n; b += kBlock) combine(acc, parts[b]);
    block_reduce_write(acc, out);
}

__global__ void fill_undrawn_kernel(tm_sample_rec* recs, u64 count) {
    const u64 r = (u64)blockIdx.x * kBlock + threadIdx.x;
    if (r >= count) return;
    tm_sample_rec& out = recs[r];
    out.interval = 0;
    out.status = 4;
    out.n_phi = 0;
    out.pad = 0;
    for (int x = 0; x < 8; ++x) out.eid[x] = -1;
    out.m_phi.lo = out.m_phi.hi = 0;
}

using SampleKernel = void (*)(SampleArgs);

template <typename W, bool kCount, bool kSorted>
SampleKernel sample_variant(const SampleArgs& a) {
    if constexpr (kSorted) {
        if (a.has_win && !a.general_runs && a.nt <= 4 && a.k <= 5)
            return sample_kernel<W, kCount, false, true, true, true>;
        if constexpr (sizeof(W) == 16) {
            if (a.has_win && !a.general_runs && !a.list_wide)
                return sample_kernel<W, kCount, false, true, true, false, true>;
        }
        if (a.has_win)
            return a.general_runs ? sample_kernel<W, kCount, true, true, true>
                                  : sample_kernel<W, kCount, false, true, true>;
    }
    return a.general_runs ? sample_kernel<W, kCount, true, kSorted, false>
                          : sample_kernel<W, kCount, false, kSorted, false>;
}

// The sampling kernel for a's plan and tables: counting variant or not,
// 64- or 128-bit weights, root-sorted order or not.
SampleKernel pick_sample(bool count, bool wide, bool sorted, const SampleArgs& a) {
    if (count) {
        if (wide) return sorted ? sample_variant<u128, true, true>(a) : sample_variant<u128, true, false>(a);
        return sorted ? sample_variant<u64, true, true>(a) : sample_variant<u64, true, false>(a);
    }
    if (wide) return sorted ? sample_variant<u128, false, true>(a) : sample_variant<u128, false, false>(a);
    return sorted ? sample_variant<u64, false, true>(a) : sample_variant<u64, false, false>(a);
}

hipError_t launch_sample(SampleKernel k, dim3 grid, size_t lds, hipStream_t st, const SampleArgs& a) {
    void* args[] = {const_cast<SampleArgs*>(&a)};
    return hipLaunchKernel(reinterpret_cast<const void*>(k), grid, dim3(kBlock), args, lds, st);
}

// Workgroups of a grid-stride sampling launch over n samples: whole rounds of
// the workgroups the chip holds at once for kernel k, since a partial last
// round leaves CUs idle while the rest finish; two rounds, six for runs of
// 2^25 samples and more (the partials' reduction is then negligible).
unsigned sample_grid(SampleKernel k, size_t lds, u64 n) {
    // a grid of at most one workgroup per CU is never more than one round
    // (the unsorted runs, below 2^16 samples, all stay there)
    const u64 need = (n + kBlock - 1) / kBlock;
    if (need <= 256) return (unsigned)std::max<u64>(1, need);
    struct Occ {
        SampleKernel k;
        size_t lds;
        int dev, resident;
    };
    static std::mutex mu;
    static std::vector<Occ> seen;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    int resident = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        for (const Occ& o : seen)
            if (o.k == k && o.lds == lds && o.dev == dev) resident = o.resident;
    }
    if (resident == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k), kBlock, lds) !=
                hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            per_cu = 0;
        }
        resident = per_cu > 0 && cus > 0 ? per_cu * cus : 1024;
        std::lock_guard<std::mutex> lk(mu);
        seen.push_back(Occ{k, lds, dev, resident});
    }
    const u64 rounds = n >= ((u64)1 << 25) ? 6 : 2;
    return (unsigned)std::min<u64>(need, rounds * (u64)resident);
}

// Samples per chunk (sort keys and offsets are 32-bit), and the smallest
// count for which sorting by root pays for itself.
constexpr u64 kChunk = (u64)1 << 28;
constexpr u64 kSortMin = (u64)1 << 16;

int bits_of(u64 x) {
    int b = 0;
    while (x) { ++b; x >>= 1; }
    return b;
}

// The lowest root-key bit the root sort looks at.  The sort only groups
// samples by root for locality (no result depends on the order), so up to
// six low bits (samples within 32 list positions) stay unsorted when that
// saves a pass.
int root_sort_lo_bit(int key_bits) {
    // whole 8-bit digits: at 1e7 keys a 9-bit digit leaves too few keys per
    // digit in a tile for its writes to stay contiguous
    const int need = key_bits > 6 ? key_bits - 6 : 0;
    const int passes = (need + 7) / 8;
    const int lo = key_bits - passes * 8;
    return lo > 0 ? lo : 0;
}

// Per-job kernel arguments from a weight set (everything but the sample range).
void fill_args(const tm_weights* w, SampleArgs* out, size_t* lds_out) {
    const HostPlan& P = w->plan;
    SampleArgs& a = *out;
    std::memset(&a, 0, sizeof a);
    a.G = w->g->d;
    a.delta = P.mo.delta;
    a.ilen = w->ilen;
    a.exclude = (w->constraints & TM_C_EXCLUDE) ? 1 : 0;
    a.q = w->q;
    a.k = P.mo.k;
    a.nt = P.nt;
    for (int s = 0; s < P.nt; ++s) {
        const int e = P.edge[s];
        a.esrc[s] = P.mo.src[e];
        a.edst[s] = P.mo.dst[e];
        a.parent[s] = P.parent[s];
        a.side[s] = P.side[s];
        a.dir[s] = P.alpha[s] > 0 ? 0 : 1;
        a.beta[s] = P.beta[s];
        a.leaf[s] = P.n_children[s] == 0;
        a.new_vertex[s] = P.new_vertex[s];
        if (s > 0) {
            const int pe = P.edge[P.parent[s]];
            a.gv[s] = P.side[s] ? P.mo.dst[pe] : P.mo.src[pe];
            a.ov[s] = P.side[s] ? P.mo.src[pe] : P.mo.dst[pe];
        }
        a.by_pi[s] = P.by_pi[s];
        a.pi_pos[P.by_pi[s]] = s;
        a.same_window[s] = P.same_window[s];
        for (int par = 0; par < 2; ++par) {
            a.qt[s][par] = w->qt[s][par];
            a.qn[s][par] = w->qn[s][par];
            a.qtc[s][par] = w->qtc[s][par];
            a.win[s][par] = w->win[s][par];
        }
        // the list slot s's parent is drawn from (the root list for the center)
        if (s > 0) a.win_from[s] = P.parent[s] == 0 ? P.root_dir : (P.alpha[P.parent[s]] > 0 ? 0 : 1);
    }
    a.has_win = w->has_win ? 1 : 0;
    a.list_wide = w->list_wide ? 1 : 0;
    a.root_dir = P.root_dir;
    a.qc[0] = w->qc[0];
    a.qc[1] = w->qc[1];
    a.ilo = w->ilo;
    a.ihi = w->ihi;
    a.cumW = w->cumW;
    a.guide = w->guide;
    a.guide_bits = w->guide_bits;
    a.ioff = w->ioff;
    const size_t wsz = w->wide ? 16 : 8;
    const size_t cum_bytes = (size_t)(w->q + 1) * wsz;
    // with a guide a draw reads one or two prefix entries: no staging
    a.cum_in_lds = !w->guide && cum_bytes <= (size_t)kCumLdsBytes;
    const size_t lds = a.cum_in_lds ? cum_bytes : 0;
    a.W_lo = (u64)w->W;
    a.W_hi = (u64)(w->W >> 64);
    a.n_free = P.n_free;
    for (int f = 0; f < P.n_free; ++f) {
        a.free_src[f] = P.free_src[f];
        a.free_dst[f] = P.free_dst[f];
    }
    a.n_runs = P.n_runs;
    bool has_lead = false, has_trail = false;
    for (int r = 0; r < P.n_runs; ++r) {
        a.run_first[r] = P.run_first[r];
        a.run_len[r] = P.run_len[r];
        a.run_prev[r] = P.run_prev[r];
        a.run_next[r] = P.run_next[r];
        if (P.run_len[r] > 2) a.general_runs = 1;
        if (P.run_prev[r] < 0) has_lead = true;
        if (P.run_next[r] < 0) has_trail = true;
    }
    if (has_lead && has_trail) a.general_runs = 1;
    if (P.po) {
        // a partial order completes in the general variant, by its own counter
        a.general_runs = 1;
        a.po = 1;
        for (int s = 0; s < kMaxSlots; ++s) a.po_tpred[s] = P.po_tpred[s];
        for (int f = 0; f < kPoMaxFree; ++f) {
            a.po_f_tpred[f] = P.po_f_tpred[f];
            a.po_f_tsucc[f] = P.po_f_tsucc[f];
            a.po_f_fpred[f] = P.po_f_fpred[f];
        }
    }
    *lds_out = lds;
}

// ---------------------------------------------------------------------------
// Batched sampling: many jobs (weight sets) in one pass.  Every sample of
// every job gets a root key prefixed by its job, one radix sort orders them
// all, and persistent kernels pull (job, range) tiles from a device counter.
// ---------------------------------------------------------------------------
struct Tile {
    int32_t job;
    int32_t pad;
    u64 begin, end;  // sample offsets (roots) or sorted positions (samples) of the job
    u64 out;         // roots: where the job's keys start in the batch arrays
};

template <typename W>
__global__ void __launch_bounds__(kBlock)
batch_root_kernel(const SampleArgs* __restrict__ jobs, const Tile* __restrict__ tiles, int n_tiles,
                  int* __restrict__ counter, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                  int* __restrict__ ovf) {
    extern __shared__ unsigned char lds_raw[];
    __shared__ int s_tile;
    bool bad = false;
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) s_tile = atomicAdd(counter, 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_tile);  // uniform: job fields load as scalars
        if (t >= n_tiles) break;
        const Tile T = tiles[t];
        const SampleArgs& a = jobs[T.job];
        const W Wtot = a.Wdev ? *static_cast<const W*>(a.Wdev) : (W)(((u128)a.W_hi << 64) | a.W_lo);
        if ((a.wflag && *a.wflag != 0) || Wtot == 0) {
            // a skipped job keeps valid keys; its samples are not drawn
            for (u64 r = T.begin + threadIdx.x; r < T.end; r += kBlock) {
                keys[T.out + r] = a.key_base;
                vals[T.out + r] = (uint32_t)r;
            }
            continue;
        }
        const W* cumG = static_cast<const W*>(a.cumW);
        const int32_t ncum = (int32_t)a.q + 1;
        W* cumL = reinterpret_cast<W*>(lds_raw);
        if (a.cum_in_lds) {
            for (int32_t x = threadIdx.x; x < ncum; x += kBlock) cumL[x] = cumG[x];
            __syncthreads();
        }
        const W* cum = a.cum_in_lds ? cumL : cumG;
        for (u64 r = T.begin + threadIdx.x; r < T.end; r += kBlock) {
            const X128 X = draw_block(a.seed, a.j0 + r, 0);
            RootGuide g0, g1;
            guide_pair(a, X, g0, g1);
            keys[T.out + r] = a.key_base + root_key<W>(a, cum, Wtot, X, g0, g1, bad);
            vals[T.out + r] = (uint32_t)r;
        }
    }
    if (bad) atomicOr(ovf, 2);
}

// kWinMode: 0 no job kept its child windows, 1 every job did, 2 some did
// (each path is compiled only where it can run: registers set occupancy).
template <typename W, bool kGeneral, int kWinMode>
__global__ void __launch_bounds__(kBlock)
batch_sample_kernel(const SampleArgs* __restrict__ jobs, const Tile* __restrict__ tiles, int n_tiles,
                    int* __restrict__ counter, Partial* __restrict__ tile_parts, int* __restrict__ ovf) {
    __shared__ int s_tile;
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) s_tile = atomicAdd(counter, 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_tile);  // uniform: job fields load as scalars
        if (t >= n_tiles) break;
        const Tile T = tiles[t];
        const SampleArgs& a = jobs[T.job];
        LaneAcc L = lane_zero();
        const bool skip = (a.wflag && *a.wflag != 0) || (a.Wdev && *static_cast<const W*>(a.Wdev) == 0);
        if (!skip) {
            if (kWinMode == 1 || (kWinMode == 2 && a.has_win))
                sample_positions<W, false, kGeneral, true, kWinMode != 0>(a, a, nullptr, T.begin + threadIdx.x,
                                                                          T.end, kBlock, L);
            else
                sample_positions<W, false, kGeneral, true, false>(a, a, nullptr, T.begin + threadIdx.x, T.end, kBlock, L);
        }
        lanes_reduce(L, &tile_parts[t], ovf);
    }
}

template <typename W, bool kGeneral>
void launch_batch_sample(int mode, dim3 grid, hipStream_t st, const SampleArgs* jobs, const Tile* tiles, int n_tiles,
                         int* counter, Partial* tile_parts, int* ovf) {
    if (mode == 0)
        hipLaunchKernelGGL((batch_sample_kernel<W, kGeneral, 0>), grid, dim3(kBlock), 0, st, jobs, tiles, n_tiles,
                           counter, tile_parts, ovf);
    else if (mode == 1)
        hipLaunchKernelGGL((batch_sample_kernel<W, kGeneral, 1>), grid, dim3(kBlock), 0, st, jobs, tiles, n_tiles,
                           counter, tile_parts, ovf);
    else
        hipLaunchKernelGGL((batch_sample_kernel<W, kGeneral, 2>), grid, dim3(kBlock), 0, st, jobs, tiles, n_tiles,
                           counter, tile_parts, ovf);
}

// One block per job: the sum of the job's tile partials.
__global__ void __launch_bounds__(kBlock)
job_reduce_kernel(const Partial* tile_parts, const int* first, const int* count, Partial* out) {
    Partial acc;
    acc.acc2 = 0;
    acc.acc2_sq = 0;
    acc.n_valid = acc.n_vertex = acc.n_delta = acc.n_order = acc.n_nonzero = 0;
    acc.flags = 0;
    acc.bytes = 0;
    const int f = first[blockIdx.x], c = count[blockIdx.x];
    for (int b = threadIdx.x; b < c; b += kBlock) combine(acc, tile_parts[f + b]);
    block_reduce_write(acc, &out[blockIdx.x]);
}

// Random instance listing: for every valid record with 0 < M_phi <= kListMax,
// the r-th completion (r from draw kListDraw of the sample) by a depth-first
// walk over the motif edges in pi order -- tree edges fixed, non-tree edges
// over their multi-edge lists within delta of the tree times, in eid order --
// with strictly increasing times and everything within delta of the first.
constexpr uint32_t kListDraw = 15;
constexpr u64 kListMax = (u64)1 << 20;

struct ListArgs {
    int l;
    int kind[TM_MAX_L];  // motif edge in pi order: its tree slot, or -1 - (its index among the non-tree edges)
};

__global__ void __launch_bounds__(kBlock)
list_kernel(SampleArgs a, ListArgs la, const tm_sample_rec* recs, u64 count, int32_t* out) {
    constexpr int NT = kMaxSlots - 1;
    const DevGraph& G = a.G;
    const u64 tmask = tmask_of(G);
    for (u64 r = (u64)blockIdx.x * kBlock + threadIdx.x; r < count; r += (u64)gridDim.x * kBlock) {
        int32_t* row = out + r * TM_MAX_L;
        for (int p = 0; p < TM_MAX_L; ++p) row[p] = -1;
        const tm_sample_rec& rec = recs[r];
        const u128 m = ((u128)rec.m_phi.hi << 64) | rec.m_phi.lo;
        if (rec.status != 0 || m == 0 || m > (u128)kListMax) continue;
        int32_t img[TM_MAX_K];
        int64_t tslot[NT];
        int32_t eslot[NT];
        for (int x = 0; x < TM_MAX_K; ++x) img[x] = -1;
        int64_t tmin = 0, tmax = 0;
        for (int x = 0; x < a.nt; ++x) {
            const int s = a.by_pi[x];
            const int32_t e = rec.eid[x];
            tslot[s] = G.t[e];
            eslot[s] = e;
            img[a.esrc[s]] = G.src[e];
            img[a.edst[s]] = G.dst[e];
            tmin = x == 0 || G.t[e] < tmin ? G.t[e] : tmin;
            tmax = x == 0 || G.t[e] > tmax ? G.t[e] : tmax;
        }
        // candidate ranges: tree edges one entry, non-tree edges a run of the
        // N order of the source's out-list
        int32_t beg[TM_MAX_L], end[TM_MAX_L], pos[TM_MAX_L], pick_e[TM_MAX_L];
        int64_t tt[TM_MAX_L];
        for (int p = 0; p < la.l; ++p) {
            if (la.kind[p] >= 0) {
                beg[p] = 0;
                end[p] = 1;
            } else {
                const int f = -1 - la.kind[p];
                const int32_t x = img[a.free_src[f]], y = img[a.free_dst[f]];
                int32_t lo, hi;
                el_run_dir(G, 0, x, y, tmax - a.delta, tmin + a.delta, G.off[0][x], G.off[0][x + 1], beg[p], end[p],
                           lo, hi);
            }
        }
        u128 rank = scale(draw_block(a.seed, a.j0 + r, kListDraw), m);
        int p = 0;
        pos[0] = beg[0];
        bool found = false;
        while (p >= 0) {
            if (pos[p] >= end[p]) {
                --p;
                if (p >= 0) ++pos[p];
                continue;
            }
            int64_t t;
            int32_t e;
            if (la.kind[p] >= 0) {
                t = tslot[la.kind[p]];
                e = eslot[la.kind[p]];
            } else {
                t = (int64_t)(G.nkey[0][pos[p]] & tmask);
                e = G.neid[0][pos[p]];
            }
            if (p > 0 && t <= tt[p - 1]) {
                ++pos[p];
                continue;
            }
            if (p > 0 && t - tt[0] > a.delta) {
                pos[p] = end[p];  // later entries are later in time
                continue;
            }
            tt[p] = t;
            pick_e[p] = e;
            if (p == la.l - 1) {
                if (rank == 0) {
                    found = true;
                    break;
                }
                --rank;
                ++pos[p];
                continue;
            }
            ++p;
            pos[p] = beg[p];
        }
        if (found)
            for (int q = 0; q < la.l; ++q) row[q] = pick_e[q];
    }
}

}  // namespace

int sample_run(tm_weights* w, u64 seed, u64 j0, u64 count, u64 k_total, hipStream_t st,
               tm_result* out, tm_sample_rec* recs, u64* model_bytes, const int* wflag, bool* overflowed) {
    if (model_bytes) {
        *model_bytes = 0;
        recs = nullptr;
    }
    // enqueued after a 64-bit build the host has not waited for: W is read
    // from the table with the sums, and the kernels draw nothing when the
    // build overflowed (*wflag) or W is 0
    const bool deferred = wflag != nullptr;
    if (deferred && (recs || model_bytes || count == 0 || w->wide))
        return tm_fail(TM_EINVAL, "sample: a deferred run takes samples and nothing else");
    if (overflowed) *overflowed = false;
    const HostPlan& P = w->plan;
    std::memset(out, 0, sizeof *out);
    out->k = k_total;
    out->q = w->q;
    out->W.lo = (u64)w->W;
    out->W.hi = (u64)(w->W >> 64);
    if (w->wide) out->flags |= TM_F_WIDE;
    if (!deferred && (w->W == 0 || count == 0)) {
        if (w->W == 0) out->flags |= TM_F_W_ZERO;
        if (recs && count) {
            hipLaunchKernelGGL(fill_undrawn_kernel, dim3((unsigned)((count + kBlock - 1) / kBlock)),
                               dim3(kBlock), 0, st, recs, count);
            TM_HIP(hipGetLastError());
            TM_HIP(sync_stream(st));
        }
        return TM_OK;
    }
    if (P.nt < 1 || P.nt > 7) return tm_fail(TM_EINVAL, "sample: tree with %d edges", P.nt);
    SampleArgs a;
    size_t lds = 0;
    fill_args(w, &a, &lds);
    a.seed = seed;
    a.key_base = 0;
    const bool sorted = count >= kSortMin;
    const u64 chunk = std::min<u64>(count, kChunk);
    // the sorted variant does not search the interval prefix (no LDS copy)
    const SampleKernel kfn = pick_sample(model_bytes != nullptr, w->wide, sorted, a);
    const size_t klds = sorted ? 0 : lds;
    const int blocks = (int)sample_grid(kfn, klds, chunk);
    const int key_bits = bits_of(2 * (u64)w->g->m - 1);
    Partial* parts = nullptr;
    int* ovf = nullptr;
    uint32_t *k0 = nullptr, *v0 = nullptr, *k1 = nullptr, *v1 = nullptr;
    TM_HIP(dev_alloc((void**)&parts, (size_t)(blocks + 1) * sizeof(Partial), st));
    TM_HIP(dev_alloc((void**)&ovf, sizeof(int), st));
    TM_TRY(fill_u32(ovf, 1, 0u, st));
    if (sorted) {
        TM_HIP(dev_alloc((void**)&k0, chunk * sizeof(uint32_t), st));
        TM_HIP(dev_alloc((void**)&v0, chunk * sizeof(uint32_t), st));
        TM_HIP(dev_alloc((void**)&k1, chunk * sizeof(uint32_t), st));
        TM_HIP(dev_alloc((void**)&v1, chunk * sizeof(uint32_t), st));
    }
    a.parts = parts;
    a.ovf = ovf;
    u64 hW = 0;
    int hflag = 0;
    if (deferred) {
        a.Wdev = static_cast<const unsigned char*>(w->cumW) + w->q * sizeof(u64);
        a.wflag = wflag;
    }
    Partial h;
    std::memset(&h, 0, sizeof h);
    int hovf = 0;
    for (u64 c0 = 0; c0 < count; c0 += chunk) {
        const u64 n = std::min<u64>(chunk, count - c0);
        a.j0 = j0 + c0;
        a.count = n;
        a.recs = recs ? recs + c0 : nullptr;
        const dim3 grid((unsigned)std::min<u64>((n + kBlock - 1) / kBlock, (u64)blocks));
        // the root draws keep a wider grid (more draws in flight)
        const dim3 rgrid((unsigned)std::min<u64>((n + kBlock - 1) / kBlock, 8192));
        StageTimer t_roots, t_sample, t_reduce;
        if (sorted) {
            if (!model_bytes) t_roots.start(TM_STAGE_ROOTS, st);
            if (w->wide)
                hipLaunchKernelGGL(root_kernel<u128>, rgrid, dim3(kBlock), lds, st, a, k0, v0);
            else
                hipLaunchKernelGGL(root_kernel<u64>, rgrid, dim3(kBlock), lds, st, a, k0, v0);
            TM_HIP(hipGetLastError());
            uint32_t *ks, *vs;
            TM_TRY(radix_sort_pairs<uint32_t>(k0, v0, k1, v1, (int64_t)n, root_sort_lo_bit(key_bits), key_bits, &ks,
                                              &vs, ovf, st, true));
            a.skey = ks;
            a.sval = vs;
            t_roots.stop();
        }
        if (!model_bytes) t_sample.start(TM_STAGE_SAMPLE, st);
        TM_HIP(launch_sample(kfn, grid, klds, st, a));
        t_sample.stop();
        if (!model_bytes) t_reduce.start(TM_STAGE_REDUCE, st);
        hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kBlock), 0, st, (const Partial*)parts,
                           (int)grid.x, parts + blocks);
        TM_HIP(hipGetLastError());
        t_reduce.stop();
        Partial hc;
        TM_HIP(read_back({{&hc, parts + blocks, sizeof hc},
                          {&hovf, ovf, sizeof hovf},
                          {&hflag, wflag, deferred ? sizeof hflag : 0},
                          {&hW, a.Wdev, deferred ? sizeof hW : 0}},
                         st));
        t_roots.finish();
        t_sample.finish();
        t_reduce.finish();
        if (hovf) break;
        if (deferred && (hflag || hW == 0)) break;  // nothing was drawn
        if (!add_ok(h.acc2, hc.acc2, &h.acc2)) h.flags |= 1;
        if (!add_ok(h.acc2_sq, hc.acc2_sq, &h.acc2_sq)) {
            h.acc2_sq = ~(u128)0;
            h.flags |= 2;
        }
        h.n_valid += hc.n_valid;
        h.n_vertex += hc.n_vertex;
        h.n_delta += hc.n_delta;
        h.n_order += hc.n_order;
        h.n_nonzero += hc.n_nonzero;
        h.flags |= hc.flags;
        h.bytes += hc.bytes;
    }
    TM_HIP(dev_free(parts, st));
    TM_HIP(dev_free(ovf, st));
    if (sorted) {
        TM_HIP(dev_free(k0, st));
        TM_HIP(dev_free(v0, st));
        TM_HIP(dev_free(k1, st));
        TM_HIP(dev_free(v1, st));
    }
    if (model_bytes) *model_bytes = h.bytes;
    if (deferred) {
        if (hflag) {
            // the 64-bit tables overflowed: the caller builds them again
            if (overflowed) *overflowed = true;
            return TM_OK;
        }
        w->W = hW;
        out->W.lo = hW;
        out->W.hi = 0;
        if (hW == 0) {
            out->flags |= TM_F_W_ZERO;
            return TM_OK;
        }
    }
    if (hovf & kSortStall) return tm_fail(TM_EDEVICE, "sample: root sort look-back stalled");
    if (hovf & 2) return tm_fail(TM_EDEVICE, "sample: inconsistent weight tables");
    if (hovf || (h.flags & 1)) return tm_fail(TM_EOVERFLOW, "sample: a count reaches 2^128");
    out->acc2.lo = (u64)h.acc2;
    out->acc2.hi = (u64)(h.acc2 >> 64);
    out->acc2_sq.lo = (u64)h.acc2_sq;
    out->acc2_sq.hi = (u64)(h.acc2_sq >> 64);
    out->n_valid = h.n_valid;
    out->n_bad_vertex = h.n_vertex;
    out->n_bad_delta = h.n_delta;
    out->n_bad_order = h.n_order;
    out->n_nonzero = h.n_nonzero;
    if (h.flags & 2) out->flags |= TM_F_SQ_SATURATED;
    return TM_OK;
}

// ---------------------------------------------------------------------------
// Host side of batched sampling.
// ---------------------------------------------------------------------------
BatchConfig g_batch_config = {8192, 0, 0, kCumLdsBytes};

void sums_merge(JobSums& into, const JobSums& x) {
    if (!add_ok(into.acc2, x.acc2, &into.acc2)) into.flags |= 1;
    if (!add_ok(into.acc2_sq, x.acc2_sq, &into.acc2_sq)) {
        into.acc2_sq = ~(u128)0;
        into.flags |= 2;
    }
    into.n_valid += x.n_valid;
    into.n_vertex += x.n_vertex;
    into.n_delta += x.n_delta;
    into.n_order += x.n_order;
    into.n_nonzero += x.n_nonzero;
    into.flags |= x.flags;
    if (into.status == TM_OK) into.status = x.status;
}

void sums_to_result(const JobSums& h, tm_result* o) {
    o->acc2.lo = (u64)h.acc2;
    o->acc2.hi = (u64)(h.acc2 >> 64);
    o->acc2_sq.lo = (u64)h.acc2_sq;
    o->acc2_sq.hi = (u64)(h.acc2_sq >> 64);
    o->n_valid = h.n_valid;
    o->n_bad_vertex = h.n_vertex;
    o->n_bad_delta = h.n_delta;
    o->n_bad_order = h.n_order;
    o->n_nonzero = h.n_nonzero;
    if (h.flags & 2) o->flags |= TM_F_SQ_SATURATED;
    o->status = (h.flags & 1) ? TM_EOVERFLOW : h.status;
}

namespace {

// One batched pass over jobs whose root-key ranges and sample offsets all fit
// 32 bits together: job y's keys are key_base[y] + (its root key < 2 m_y).
// One batched pass over jobs act: host arrays, device buffers, launches.
struct Group {
    int na = 0;
    u64 total = 0;
    int key_bits = 1, passes = 1, blocks = 0;
    size_t root_lds = 0;
    std::vector<SampleArgs> args;
    std::vector<Tile> rt, stt;
    std::vector<int> g_rt_first, g_st_first, jfirst, jcount;
    int g_win[4] = {0, 0, 0, 0};  // per kernel group: the batch_sample_kernel window mode
    SampleArgs* djobs = nullptr;
    Tile *drt = nullptr, *dst = nullptr;
    uint32_t *k0 = nullptr, *v0 = nullptr, *k1 = nullptr, *v1 = nullptr;
    Partial *tparts = nullptr, *jparts = nullptr;
    int *ctr = nullptr, *ovf = nullptr, *djf = nullptr, *djc = nullptr;
    unsigned char* pinned = nullptr;  // captured passes: host staging of the uploads
};

// Host side: job arguments, tiles grouped by kernel variant.  Wdev / wflag
// (per job in act, may be null) switch on the captured form.
void group_prepare(tm_weights* const* ws, const std::vector<int>& act, const u64* j0s, const u64* counts,
                   const u64* seeds, const BatchConfig& cfg, const void* const* Wdev, const int* const* wflag,
                   Group& G) {
    const int na = (int)act.size();
    G.na = na;
    u64 key_space = 0;
    std::vector<uint32_t> key_base(na);
    for (int y = 0; y < na; ++y) {
        key_base[y] = (uint32_t)key_space;
        key_space += 2 * (u64)ws[act[y]]->g->m;
        G.total += counts[act[y]];
    }
    G.key_bits = std::max(1, bits_of(key_space - 1));
    G.passes = radix_passes(G.key_bits - root_sort_lo_bit(G.key_bits));
    const int tile = cfg.tile > 0 ? cfg.tile : 8192;
    int cus = 256;
    {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            cus = prop.multiProcessorCount;
    }
    G.blocks = cfg.blocks > 0 ? cfg.blocks : 8 * cus;
    G.args.resize(na);
    std::vector<u64> base(na);
    u64 off = 0;
    for (int y = 0; y < na; ++y) {
        size_t lds;
        fill_args(ws[act[y]], &G.args[y], &lds);
        G.args[y].seed = seeds[act[y]];
        G.args[y].j0 = j0s[act[y]];
        G.args[y].count = counts[act[y]];
        G.args[y].key_base = key_base[y];
        G.args[y].Wdev = Wdev ? Wdev[y] : nullptr;
        G.args[y].wflag = wflag ? wflag[y] : nullptr;
        // the root draws stage the interval prefix in LDS when it fits the
        // configured size (jobs with a root guide read one or two entries)
        const tm_weights* wy = ws[act[y]];
        const size_t cum_bytes = (size_t)(wy->q + 1) * (wy->wide ? 16 : 8);
        G.args[y].cum_in_lds = !wy->guide && cum_bytes <= (size_t)cfg.root_lds;
        if (G.args[y].cum_in_lds) G.root_lds = (size_t)cfg.root_lds;
        base[y] = off;
        off += counts[act[y]];
    }
    G.g_rt_first.assign(5, 0);
    G.g_st_first.assign(5, 0);
    G.jfirst.assign(na, 0);
    G.jcount.assign(na, 0);
    for (int grp = 0; grp < 4; ++grp) {
        G.g_rt_first[grp] = (int)G.rt.size();
        G.g_st_first[grp] = (int)G.stt.size();
        int with = 0, without = 0;
        for (int y = 0; y < na; ++y) {
            const tm_weights* w = ws[act[y]];
            const int gy = (w->wide ? 2 : 0) + (G.args[y].general_runs ? 1 : 0);
            if (gy != grp) continue;
            if (G.args[y].has_win) ++with; else ++without;
            G.jfirst[y] = (int)G.stt.size();
            const u64 cy = counts[act[y]];
            for (u64 b = 0; b < cy; b += (u64)tile) {
                const u64 e = std::min<u64>(cy, b + (u64)tile);
                G.rt.push_back(Tile{y, 0, b, e, base[y]});
                G.stt.push_back(Tile{y, 0, base[y] + b, base[y] + e, 0});
            }
            G.jcount[y] = (int)G.stt.size() - G.jfirst[y];
        }
        G.g_win[grp] = with == 0 ? 0 : (without == 0 ? 1 : 2);
    }
    G.g_rt_first[4] = (int)G.rt.size();
    G.g_st_first[4] = (int)G.stt.size();
}

int group_alloc(Group& G, hipStream_t st) {
    const int na = G.na;
    TM_HIP(dev_alloc((void**)&G.djobs, na * sizeof(SampleArgs), st));
    TM_HIP(dev_alloc((void**)&G.drt, G.rt.size() * sizeof(Tile), st));
    TM_HIP(dev_alloc((void**)&G.dst, G.stt.size() * sizeof(Tile), st));
    TM_HIP(dev_alloc((void**)&G.k0, G.total * sizeof(uint32_t), st));
    TM_HIP(dev_alloc((void**)&G.v0, G.total * sizeof(uint32_t), st));
    TM_HIP(dev_alloc((void**)&G.k1, G.total * sizeof(uint32_t), st));
    TM_HIP(dev_alloc((void**)&G.v1, G.total * sizeof(uint32_t), st));
    TM_HIP(dev_alloc((void**)&G.tparts, G.stt.size() * sizeof(Partial), st));
    TM_HIP(dev_alloc((void**)&G.jparts, na * sizeof(Partial), st));
    TM_HIP(dev_alloc((void**)&G.ctr, 16 * sizeof(int), st));
    TM_HIP(dev_alloc((void**)&G.ovf, sizeof(int), st));
    TM_HIP(dev_alloc((void**)&G.djf, na * sizeof(int), st));
    TM_HIP(dev_alloc((void**)&G.djc, na * sizeof(int), st));
    // the sorted arrays end where an even number of passes leaves them
    for (int y = 0; y < na; ++y) {
        G.args[y].skey = G.passes % 2 == 0 ? G.k0 : G.k1;
        G.args[y].sval = G.passes % 2 == 0 ? G.v0 : G.v1;
    }
    return TM_OK;
}

// Uploads of the host arrays; staged through pinned memory when `pinned`
// (captured passes replay the copies from that buffer).
int group_upload(Group& G, bool pinned, hipStream_t st) {
    const size_t sz[5] = {G.na * sizeof(SampleArgs), G.rt.size() * sizeof(Tile), G.stt.size() * sizeof(Tile),
                          G.na * sizeof(int), G.na * sizeof(int)};
    const void* src[5] = {G.args.data(), G.rt.data(), G.stt.data(), G.jfirst.data(), G.jcount.data()};
    void* dst[5] = {G.djobs, G.drt, G.dst, G.djf, G.djc};
    if (pinned) {
        size_t total = 0;
        for (size_t b : sz) total += (b + 255) & ~(size_t)255;
        TM_HIP(hipHostMalloc((void**)&G.pinned, total, hipHostMallocDefault));
        size_t o = 0;
        for (int x = 0; x < 5; ++x) {
            std::memcpy(G.pinned + o, src[x], sz[x]);
            src[x] = G.pinned + o;
            o += (sz[x] + 255) & ~(size_t)255;
        }
    }
    for (int x = 0; x < 5; ++x)
        if (sz[x]) TM_HIP(hipMemcpyAsync(dst[x], src[x], sz[x], hipMemcpyHostToDevice, st));
    return TM_OK;
}

// Counters, root draws, the sort, sampling and per-job sums into jparts.
int group_launch(Group& G, hipStream_t st, bool timed) {
    TM_TRY(fill_u32(G.ctr, 16, 0u, st));
    TM_TRY(fill_u32(G.ovf, 1, 0u, st));
    StageTimer t_roots, t_sample, t_reduce;
    if (timed) t_roots.start(TM_STAGE_ROOTS, st);
    for (int grp = 0; grp < 4; ++grp) {
        const int nt = G.g_rt_first[grp + 1] - G.g_rt_first[grp];
        if (nt == 0) continue;
        const dim3 grid((unsigned)std::min(G.blocks, nt));
        const Tile* tl = G.drt + G.g_rt_first[grp];
        if (grp >= 2)
            hipLaunchKernelGGL(batch_root_kernel<u128>, grid, dim3(kBlock), G.root_lds, st, G.djobs, tl, nt,
                               G.ctr + grp, G.k0, G.v0, G.ovf);
        else
            hipLaunchKernelGGL(batch_root_kernel<u64>, grid, dim3(kBlock), G.root_lds, st, G.djobs, tl, nt,
                               G.ctr + grp, G.k0, G.v0, G.ovf);
        TM_HIP(hipGetLastError());
    }
    {
        uint32_t *ksr, *vsr;
        TM_TRY(radix_sort_pairs<uint32_t>(G.k0, G.v0, G.k1, G.v1, (int64_t)G.total, root_sort_lo_bit(G.key_bits),
                                          G.key_bits, &ksr, &vsr,
                                          G.ovf, st));
        if (ksr != G.args[0].skey) return tm_fail(TM_EDEVICE, "batch: unexpected sort buffer");
    }
    t_roots.stop();
    if (timed) t_sample.start(TM_STAGE_SAMPLE, st);
    for (int grp = 0; grp < 4; ++grp) {
        const int nt = G.g_st_first[grp + 1] - G.g_st_first[grp];
        if (nt == 0) continue;
        const dim3 grid((unsigned)std::min(G.blocks, nt));
        const Tile* tl = G.dst + G.g_st_first[grp];
        Partial* tp = G.tparts + G.g_st_first[grp];
        int* c = G.ctr + 4 + grp;
        const int wm = G.g_win[grp];
        switch (grp) {
            case 0: launch_batch_sample<u64, false>(wm, grid, st, G.djobs, tl, nt, c, tp, G.ovf); break;
            case 1: launch_batch_sample<u64, true>(wm, grid, st, G.djobs, tl, nt, c, tp, G.ovf); break;
            case 2: launch_batch_sample<u128, false>(wm, grid, st, G.djobs, tl, nt, c, tp, G.ovf); break;
            default: launch_batch_sample<u128, true>(wm, grid, st, G.djobs, tl, nt, c, tp, G.ovf); break;
        }
        TM_HIP(hipGetLastError());
    }
    t_sample.stop();
    if (timed) t_reduce.start(TM_STAGE_REDUCE, st);
    hipLaunchKernelGGL(job_reduce_kernel, dim3(G.na), dim3(kBlock), 0, st, (const Partial*)G.tparts,
                       (const int*)G.djf, (const int*)G.djc, G.jparts);
    TM_HIP(hipGetLastError());
    t_reduce.stop();
    if (timed) {
        TM_HIP(sync_stream(st));
        t_roots.finish();
        t_sample.finish();
        t_reduce.finish();
    }
    return TM_OK;
}

void group_free(Group& G, hipStream_t st) {
    for (void* q : {(void*)G.djobs, (void*)G.drt, (void*)G.dst, (void*)G.k0, (void*)G.v0, (void*)G.k1, (void*)G.v1,
                    (void*)G.tparts, (void*)G.jparts, (void*)G.ctr, (void*)G.ovf, (void*)G.djf, (void*)G.djc})
        (void)dev_free(q, st);
    if (G.pinned) (void)hipHostFree(G.pinned);
    G.pinned = nullptr;
}

// Per-job sums from a finished group (stream synchronised).
int group_read(Group& G, const std::vector<int>& act, hipStream_t st, JobSums* out) {
    std::vector<Partial> hp(G.na);
    int hovf = 0;
    TM_HIP(read_back({{hp.data(), G.jparts, G.na * sizeof(Partial)}, {&hovf, G.ovf, sizeof(int)}}, st));
    if (hovf & kSortStall) return tm_fail(TM_EDEVICE, "batch: root sort look-back stalled");
    if (hovf & 2) return tm_fail(TM_EDEVICE, "batch: inconsistent weight tables");
    for (int y = 0; y < G.na; ++y) {
        const Partial& h = hp[y];
        JobSums& o = out[act[y]];
        o = JobSums{};
        if ((hovf & 1) || (h.flags & 1)) {
            o.status = TM_EOVERFLOW;
            continue;
        }
        o.acc2 = h.acc2;
        o.acc2_sq = h.acc2_sq;
        o.n_valid = h.n_valid;
        o.n_vertex = h.n_vertex;
        o.n_delta = h.n_delta;
        o.n_order = h.n_order;
        o.n_nonzero = h.n_nonzero;
        o.flags = h.flags & 2;
    }
    return TM_OK;
}

// One batched pass over jobs whose root-key ranges and sample offsets all fit
// 32 bits together: job y's keys are key_base[y] + (its root key < 2 m_y).
int batch_group(tm_weights* const* ws, const std::vector<int>& act, const u64* j0s, const u64* counts,
                const u64* seeds, hipStream_t st, JobSums* out, const BatchConfig& cfg) {
    Group G;
    group_prepare(ws, act, j0s, counts, seeds, cfg, nullptr, nullptr, G);
    int rc = group_alloc(G, st);
    if (rc == TM_OK) rc = group_upload(G, false, st);
    if (rc == TM_OK) rc = group_launch(G, st, true);
    if (rc == TM_OK) rc = group_read(G, act, st, out);
    group_free(G, st);
    (void)sync_stream(st);
    return rc;
}

}  // namespace

int batch_sample_pass(tm_weights* const* ws, const u64* j0s, const u64* counts, const u64* seeds, int n,
                      hipStream_t st, JobSums* out, const BatchConfig& cfg) {
    std::vector<int> act;
    for (int x = 0; x < n; ++x) {
        out[x] = JobSums{};
        tm_weights* w = ws[x];
        if (w->plan.nt < 1 || w->plan.nt > 7) return tm_fail(TM_EINVAL, "batch: job %d tree size", x);
        if (w->W != 0 && counts[x] > 0) act.push_back(x);
    }
    // groups in job order whose key ranges (2 m per job) and sample counts
    // each stay below 2^32 (or the configured smaller limit); a job of 2^32
    // samples or more samples on its own
    const u64 lim = (u64)1 << 32;
    const u64 glim = cfg.group_limit > 0 && cfg.group_limit < lim ? cfg.group_limit : lim;
    std::vector<int> grp;
    u64 keys = 0, cnt = 0;
    auto flush = [&]() -> int {
        if (grp.empty()) return TM_OK;
        const int rc = batch_group(ws, grp, j0s, counts, seeds, st, out, cfg);
        grp.clear();
        keys = cnt = 0;
        return rc;
    };
    for (int x : act) {
        const u64 kx = 2 * (u64)ws[x]->g->m;
        if (counts[x] >= lim) {
            tm_result r;
            tm_sample_rec* none = nullptr;
            const int rc = sample_run(ws[x], seeds[x], j0s[x], counts[x], counts[x], st, &r, none, nullptr);
            if (rc == TM_EOVERFLOW) {
                out[x].status = rc;
                continue;
            }
            TM_TRY(rc);
            JobSums& h = out[x];
            h.acc2 = ((u128)r.acc2.hi << 64) | r.acc2.lo;
            h.acc2_sq = ((u128)r.acc2_sq.hi << 64) | r.acc2_sq.lo;
            h.n_valid = r.n_valid;
            h.n_vertex = r.n_bad_vertex;
            h.n_delta = r.n_bad_delta;
            h.n_order = r.n_bad_order;
            h.n_nonzero = r.n_nonzero;
            h.flags = (r.flags & TM_F_SQ_SATURATED) ? 2 : 0;
            continue;
        }
        if (keys + kx > glim || cnt + counts[x] >= glim) TM_TRY(flush());
        grp.push_back(x);
        keys += kx;
        cnt += counts[x];
    }
    return flush();
}

// ---------------------------------------------------------------------------
// Captured passes (recorded into a graph by the batch plan).
// ---------------------------------------------------------------------------
struct CapturedPass {
    std::vector<Group> groups;
    std::vector<std::vector<int>> acts;
    int n = 0;
};

int batch_capture_enqueue(tm_weights* const* ws, const int* const* wflag, const u64* counts, const u64* seeds,
                          int n, hipStream_t st, const BatchConfig& cfg, CapturedPass** out) {
    std::unique_ptr<CapturedPass> P(new (std::nothrow) CapturedPass());
    if (!P) return tm_fail(TM_ENOMEM, "capture: host allocation");
    P->n = n;
    const u64 lim = (u64)1 << 32;
    const u64 glim = cfg.group_limit > 0 && cfg.group_limit < lim ? cfg.group_limit : lim;
    std::vector<int> act;
    u64 keys = 0, cnt = 0;
    std::vector<u64> j0(n, 0);
    auto flush = [&]() -> int {
        if (act.empty()) return TM_OK;
        std::vector<const void*> wd(act.size());
        std::vector<const int*> wf(act.size());
        for (size_t y = 0; y < act.size(); ++y) {
            const tm_weights* w = ws[act[y]];
            wd[y] = static_cast<const unsigned char*>(w->cumW) + w->q * 8;
            wf[y] = wflag[act[y]];
        }
        P->groups.emplace_back();
        P->acts.push_back(act);
        Group& G = P->groups.back();
        group_prepare(ws, act, j0.data(), counts, seeds, cfg, wd.data(), wf.data(), G);
        TM_TRY(group_alloc(G, st));
        TM_TRY(group_upload(G, true, st));
        TM_TRY(group_launch(G, st, false));
        act.clear();
        keys = cnt = 0;
        return TM_OK;
    };
    for (int x = 0; x < n; ++x) {
        tm_weights* w = ws[x];
        if (counts[x] == 0 || w->g->m == 0 || !w->cumW) continue;
        if (w->wide) return tm_fail(TM_EINVAL, "capture: job %d has 128-bit weights", x);
        if (w->plan.nt < 1 || w->plan.nt > 7) return tm_fail(TM_EINVAL, "capture: job %d tree size", x);
        if (counts[x] >= lim) return tm_fail(TM_EINVAL, "capture: job %d draws 2^32 samples or more", x);
        const u64 kx = 2 * (u64)w->g->m;
        if (keys + kx > glim || cnt + counts[x] >= glim) {
            const int rc = flush();
            if (rc != TM_OK) {
                batch_capture_free(P.release(), st);
                return rc;
            }
        }
        act.push_back(x);
        keys += kx;
        cnt += counts[x];
    }
    const int rc = flush();
    if (rc != TM_OK) {
        batch_capture_free(P.release(), st);
        return rc;
    }
    *out = P.release();
    return TM_OK;
}

int batch_capture_read(CapturedPass* P, hipStream_t st, JobSums* out) {
    for (int x = 0; x < P->n; ++x) out[x] = JobSums{};
    for (size_t g = 0; g < P->groups.size(); ++g) TM_TRY(group_read(P->groups[g], P->acts[g], st, out));
    return TM_OK;
}

void batch_capture_free(CapturedPass* P, hipStream_t st) {
    if (!P) return;
    (void)sync_stream(st);
    for (Group& G : P->groups) group_free(G, st);
    delete P;
}

// ---------------------------------------------------------------------------
// Motif families: one tree sample stream, every member's completions.
// ---------------------------------------------------------------------------
int family_run(tm_weights* w, const HostPlan* plans, int n, u64 seed, u64 k, hipStream_t st, JobSums* sums,
               JobSums* shared) {
    for (int f = 0; f < n; ++f) sums[f] = JobSums{};
    *shared = JobSums{};
    if (w->W == 0 || k == 0) return TM_OK;
    std::vector<SampleArgs> args(n);
    size_t lds = 0;
    for (int f = 0; f < n; ++f) {
        fill_args(w, &args[f], &lds);
        args[f].seed = seed;
        const HostPlan& P = plans[f];
        // this member's non-tree edges (its tree slots are the sampled ones)
        args[f].n_free = P.n_free;
        for (int x = 0; x < P.n_free; ++x) {
            args[f].free_src[x] = P.free_src[x];
            args[f].free_dst[x] = P.free_dst[x];
        }
        args[f].n_runs = P.n_runs;
        args[f].general_runs = 0;
        bool lead = false, trail = false;
        for (int r = 0; r < P.n_runs; ++r) {
            args[f].run_first[r] = P.run_first[r];
            args[f].run_len[r] = P.run_len[r];
            args[f].run_prev[r] = P.run_prev[r];
            args[f].run_next[r] = P.run_next[r];
            if (P.run_len[r] > 2) args[f].general_runs = 1;
            lead |= P.run_prev[r] < 0;
            trail |= P.run_next[r] < 0;
        }
        if (lead && trail) args[f].general_runs = 1;
        args[f].delta = P.mo.delta;
    }
    // the tree samples are the same for every member (draws keyed by sample
    // id and slot): one root pass and sort per chunk, then one sampling pass
    // per member over the sorted roots, completing that member's non-tree
    // edges; the tree's validation counts come from the first member's pass
    const u64 chunk = std::min<u64>(k, kChunk);
    const bool sorted = chunk >= kSortMin;
    // each member's kernel and grid; the per-block partials of the widest
    // grid come first in parts, the members' reduced sums after them
    std::vector<SampleKernel> kfn(n);
    std::vector<int> fblocks(n);
    int blocks = 1;
    for (int f = 0; f < n; ++f) {
        kfn[f] = pick_sample(false, w->wide, sorted, args[f]);
        fblocks[f] = (int)sample_grid(kfn[f], sorted ? 0 : lds, chunk);
        blocks = std::max(blocks, fblocks[f]);
    }
    const int key_bits = bits_of(2 * (u64)w->g->m - 1);
    // per chunk: every member's reduced sums (after the per-block partials)
    // and flags (ovf[0] for the shared root pass and sort, ovf[1 + f] for
    // member f), read back together
    std::vector<Partial> hp(n);
    std::vector<int> hov(n + 1);
    Partial* parts = nullptr;
    int* ovf = nullptr;
    uint32_t *k0 = nullptr, *v0 = nullptr, *k1 = nullptr, *v1 = nullptr;
    TM_HIP(dev_alloc((void**)&parts, (size_t)(blocks + n) * sizeof(Partial), st));
    TM_HIP(dev_alloc((void**)&ovf, (size_t)(n + 1) * sizeof(int), st));
    if (sorted) {
        TM_HIP(dev_alloc((void**)&k0, chunk * sizeof(uint32_t), st));
        TM_HIP(dev_alloc((void**)&v0, chunk * sizeof(uint32_t), st));
        TM_HIP(dev_alloc((void**)&k1, chunk * sizeof(uint32_t), st));
        TM_HIP(dev_alloc((void**)&v1, chunk * sizeof(uint32_t), st));
    }
    int rc = TM_OK;
    for (u64 c0 = 0; c0 < k && rc == TM_OK; c0 += chunk) {
        const u64 cnt = std::min<u64>(chunk, k - c0);
        for (int f = 0; f < n; ++f) {
            args[f].j0 = c0;
            args[f].count = cnt;
            args[f].recs = nullptr;
            args[f].parts = parts;
            args[f].ovf = ovf + 1 + f;
        }
        rc = fill_u32(ovf, n + 1, 0u, st);
        if (rc != TM_OK) break;
        if (sorted) {
            const dim3 rgrid((unsigned)std::min<u64>((cnt + kBlock - 1) / kBlock, 8192));
            SampleArgs ra = args[0];
            ra.ovf = ovf;
            if (w->wide)
                hipLaunchKernelGGL(root_kernel<u128>, rgrid, dim3(kBlock), lds, st, ra, k0, v0);
            else
                hipLaunchKernelGGL(root_kernel<u64>, rgrid, dim3(kBlock), lds, st, ra, k0, v0);
            if (hipGetLastError() != hipSuccess) { rc = tm_fail(TM_EDEVICE, "family: launch"); break; }
            uint32_t *ks, *vs;
            rc = radix_sort_pairs<uint32_t>(k0, v0, k1, v1, (int64_t)cnt, root_sort_lo_bit(key_bits), key_bits, &ks,
                                            &vs, ovf, st, true);
            if (rc != TM_OK) break;
            for (int f = 0; f < n; ++f) {
                args[f].skey = ks;
                args[f].sval = vs;
            }
        }
        for (int f = 0; f < n && rc == TM_OK; ++f) {
            const dim3 grid((unsigned)std::min<u64>((cnt + kBlock - 1) / kBlock, (u64)fblocks[f]));
            if (launch_sample(kfn[f], grid, sorted ? 0 : lds, st, args[f]) != hipSuccess) {
                rc = tm_fail(TM_EDEVICE, "family: launch");
                break;
            }
            hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kBlock), 0, st, (const Partial*)parts, (int)grid.x,
                               parts + blocks + f);
            if (hipGetLastError() != hipSuccess) rc = tm_fail(TM_EDEVICE, "family: launch");
        }
        if (rc != TM_OK) break;
        if (read_back({{hp.data(), parts + blocks, (size_t)n * sizeof(Partial)},
                       {hov.data(), ovf, (size_t)(n + 1) * sizeof(int)}},
                      st) != hipSuccess) {
            rc = tm_fail(TM_EDEVICE, "family: copy");
            break;
        }
        for (int f = 0; f < n && rc == TM_OK; ++f) {
            const Partial& h = hp[f];
            const int hovf = hov[0] | hov[1 + f];
            if (hovf & (2 | kSortStall)) {
                rc = tm_fail(TM_EDEVICE, (hovf & kSortStall) ? "family: root sort look-back stalled"
                                                             : "family: inconsistent weight tables");
                break;
            }
            JobSums x;
            x.acc2 = h.acc2;
            x.acc2_sq = h.acc2_sq;
            x.n_nonzero = h.n_nonzero;
            x.flags = h.flags & 3;
            if (hovf & 1) x.flags |= 1;
            sums_merge(sums[f], x);
            if (f == 0) {
                JobSums t;
                t.n_valid = h.n_valid;
                t.n_vertex = h.n_vertex;
                t.n_delta = h.n_delta;
                t.n_order = h.n_order;
                sums_merge(*shared, t);
            }
        }
    }
    for (void* q : {(void*)parts, (void*)ovf, (void*)k0, (void*)v0, (void*)k1, (void*)v1})
        if (q) (void)dev_free(q, st);
    (void)sync_stream(st);
    return rc;
}

// ---------------------------------------------------------------------------
// Random instance listing.
// ---------------------------------------------------------------------------
int list_run(tm_weights* w, u64 seed, u64 j0, u64 count, hipStream_t st, int32_t* eids, tm_sample_rec* recs) {
    if (count == 0) return TM_OK;
    tm_sample_rec* own = nullptr;
    if (!recs) TM_HIP(dev_alloc((void**)&own, count * sizeof(tm_sample_rec), st));
    tm_sample_rec* rr = recs ? recs : own;
    tm_result res;
    int rc = sample_run(w, seed, j0, count, count, st, &res, rr, nullptr);
    if (rc == TM_OK) {
        SampleArgs a;
        size_t lds;
        fill_args(w, &a, &lds);
        a.seed = seed;
        a.j0 = j0;
        ListArgs la;
        const HostPlan& P = w->plan;
        la.l = P.mo.l;
        int nf = 0;
        for (int p = 0; p < P.mo.l; ++p) la.kind[p] = P.slot_of_edge[p] >= 0 ? P.slot_of_edge[p] : -1 - nf++;
        if (w->W == 0) {
            // nothing was drawn: every row lists nothing
            rc = fill_u32(eids, (int64_t)count * TM_MAX_L, 0xffffffffu, st);
        } else {
            const dim3 grid((unsigned)std::min<u64>((count + kBlock - 1) / kBlock, 4096));
            hipLaunchKernelGGL(list_kernel, grid, dim3(kBlock), 0, st, a, la, (const tm_sample_rec*)rr, count, eids);
            if (hipGetLastError() != hipSuccess) rc = tm_fail(TM_EDEVICE, "list: launch");
        }
    }
    if (own) (void)dev_free(own, st);
    if (sync_stream(st) != hipSuccess && rc == TM_OK) rc = tm_fail(TM_EDEVICE, "list: synchronise");
    return rc;
}

// ---------------------------------------------------------------------------
// Sampling with no allocation.  tm_sample_noalloc runs sample_run's kernels
// with every temporary -- the per-workgroup partial sums, the flag word, the
// root keys and sample offsets of the sort (two buffers each) and the sort's
// digit histograms -- carved from one file-scope device array, so it calls
// no hipMalloc, hipFree or other allocating routine.  Each device holds its
// own copy of the array until the process ends; its address on a device is
// looked up once (hipGetSymbolAddress with that device current) and used
// wherever host code needs the array: the name itself is a host-side stand-in.
// Calls on one device share that copy: calls that overlap on a device race.
// ---------------------------------------------------------------------------
namespace {

constexpr u64 kNoAllocMaxCount = (u64)1 << 21;                  // samples per call
constexpr int kNoAllocMaxBlocks = (int)(kNoAllocMaxCount / kBlock);  // sampling grid bound
constexpr size_t kNoAllocParts = (size_t)(kNoAllocMaxBlocks + 1) * sizeof(Partial);
constexpr size_t kNoAllocKeys = kNoAllocMaxCount * sizeof(uint32_t);
constexpr size_t kNoAllocHist = sort_scratch_bytes((int64_t)kNoAllocMaxCount);
constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kScratchBytes = align256(kNoAllocParts) + 256 + 4 * align256(kNoAllocKeys) + align256(kNoAllocHist);

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// The current device's copy of scratch (looked up on the first call there).
static int scratch_of_device(unsigned char** out) {
    int dev = 0;
    TM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return tm_fail(TM_EDEVICE, "sample_noalloc: device %d", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return tm_fail(TM_EDEVICE, "sample_noalloc: scratch address on device %d: %s", dev,
                           hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return TM_OK;
}

int sample_run_noalloc(tm_weights* w, u64 seed, u64 j0, u64 count, u64 k_total, hipStream_t st, tm_result* out,
                       tm_sample_rec* recs) {
    if (count > kNoAllocMaxCount)
        return tm_fail(TM_EINVAL, "sample_noalloc: %llu samples, at most %llu per call (split the id range)",
                       (unsigned long long)count, (unsigned long long)kNoAllocMaxCount);
    unsigned char* base = nullptr;
    TM_TRY(scratch_of_device(&base));
    const HostPlan& P = w->plan;
    std::memset(out, 0, sizeof *out);
    out->k = k_total;
    out->q = w->q;
    out->W.lo = (u64)w->W;
    out->W.hi = (u64)(w->W >> 64);
    if (w->wide) out->flags |= TM_F_WIDE;
    if (w->W == 0 || count == 0) {
        if (w->W == 0) out->flags |= TM_F_W_ZERO;
        if (recs && count) {
            hipLaunchKernelGGL(fill_undrawn_kernel, dim3((unsigned)((count + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                               st, recs, count);
            TM_HIP(hipGetLastError());
            TM_HIP(hipStreamSynchronize(st));
        }
        return TM_OK;
    }
    if (P.nt < 1 || P.nt > 7) return tm_fail(TM_EINVAL, "sample: tree with %d edges", P.nt);
    SampleArgs a;
    size_t lds = 0;
    fill_args(w, &a, &lds);
    a.seed = seed;
    a.key_base = 0;
    const bool sorted = count >= kSortMin;
    const SampleKernel kfn = pick_sample(false, w->wide, sorted, a);
    const size_t klds = sorted ? 0 : lds;
    // the grid of sample_run: two rounds of the kernel's occupancy (at most
    // one workgroup per 256 samples)
    const u64 need = (count + kBlock - 1) / kBlock;
    u64 blocks = need;
    if (need > 256) {
        int per_cu = 0, cus = 0, dev = 0;
        TM_HIP(hipGetDevice(&dev));
        TM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kfn), kBlock,
                                                             klds));
        TM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        const u64 resident = per_cu > 0 && cus > 0 ? (u64)per_cu * cus : 1024;
        blocks = std::min<u64>(need, 2 * resident);
    }
    blocks = std::max<u64>(1, std::min<u64>(blocks, (u64)kNoAllocMaxBlocks));
    // carve the scratch copy: partials (blocks + 1), the flag word, four key
    // and offset buffers, the sort's histograms
    Partial* parts = reinterpret_cast<Partial*>(base);
    unsigned char* at = base + align256(kNoAllocParts);
    int* ovf = reinterpret_cast<int*>(at);
    at += 256;
    uint32_t* kb[4];
    for (int x = 0; x < 4; ++x) {
        kb[x] = reinterpret_cast<uint32_t*>(at);
        at += align256(kNoAllocKeys);
    }
    uint32_t* hist = reinterpret_cast<uint32_t*>(at);
    TM_TRY(fill_u32(ovf, 1, 0u, st));  // a fill kernel: the last call's flag is stale
    a.parts = parts;
    a.ovf = ovf;
    a.j0 = j0;
    a.count = count;
    a.recs = recs;
    const dim3 grid((unsigned)blocks);
    if (sorted) {
        const int key_bits = bits_of(2 * (u64)w->g->m - 1);
        const dim3 rgrid((unsigned)std::min<u64>(need, 8192));
        if (w->wide)
            hipLaunchKernelGGL(root_kernel<u128>, rgrid, dim3(kBlock), lds, st, a, kb[0], kb[1]);
        else
            hipLaunchKernelGGL(root_kernel<u64>, rgrid, dim3(kBlock), lds, st, a, kb[0], kb[1]);
        TM_HIP(hipGetLastError());
        uint32_t *ks, *vs;
        TM_TRY(radix_sort_pairs<uint32_t>(kb[0], kb[1], kb[2], kb[3], (int64_t)count, root_sort_lo_bit(key_bits),
                                          key_bits, &ks, &vs, ovf, st, true, hist));
        a.skey = ks;
        a.sval = vs;
    }
    TM_HIP(launch_sample(kfn, grid, klds, st, a));
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kBlock), 0, st, (const Partial*)parts, (int)grid.x,
                       parts + blocks);
    TM_HIP(hipGetLastError());
    Partial h;
    int hovf = 0;
    TM_HIP(hipMemcpyAsync(&h, parts + blocks, sizeof h, hipMemcpyDeviceToHost, st));
    TM_HIP(hipMemcpyAsync(&hovf, ovf, sizeof hovf, hipMemcpyDeviceToHost, st));
    TM_HIP(hipStreamSynchronize(st));
    if (hovf & kSortStall) return tm_fail(TM_EDEVICE, "sample: root sort look-back stalled");
    if (hovf & 2) return tm_fail(TM_EDEVICE, "sample: inconsistent weight tables");
    if (hovf || (h.flags & 1)) return tm_fail(TM_EOVERFLOW, "sample: a count reaches 2^128");
    out->acc2.lo = (u64)h.acc2;
    out->acc2.hi = (u64)(h.acc2 >> 64);
    out->acc2_sq.lo = (u64)h.acc2_sq;
    out->acc2_sq.hi = (u64)(h.acc2_sq >> 64);
    out->n_valid = h.n_valid;
    out->n_bad_vertex = h.n_vertex;
    out->n_bad_delta = h.n_delta;
    out->n_bad_order = h.n_order;
    out->n_nonzero = h.n_nonzero;
    if (h.flags & 2) out->flags |= TM_F_SQ_SATURATED;
    return TM_OK;
}
