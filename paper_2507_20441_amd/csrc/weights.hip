// Preprocessing: the bottom-up spanning-tree weights (Alg. 1, Alg. 2).
//
// For a tree edge s of height h >= 1, an edge e matched to s and an interval
// I_i holding e, w_i(s, e) is the product over the children s' of s of the
// summed w_i(s', .) over the child's candidate list (Claim
// "overall-num-matches").  The candidate list is a time window of one
// vertex's out- or in-list minus the run of edges to the excluded vertex, so
// each factor is two differences of prefix sums: one along the window (T
// order), one along the excluded run (N order).  A leaf child contributes the
// plain counts.  Levels run bottom-up; after each non-center level the values
// are prefix-summed along the lists the parent searches.
//
// An edge lies in at most two intervals, i = floor(t/delta) and the one
// before, and those have different parities; so each table holds, per eid,
// one value per interval parity.  A window inside I_i only holds edges of
// blocks i and i+1, whose values for interval i are exactly the entries of
// parity i & 1 -- one prefix array per parity serves every interval.
#include <algorithm>
#include <cstring>
#include <memory>
#include <type_traits>
#include <vector>

#include "tm_primitives.h"

namespace {

struct ChildDesc {
    int side;     // 0: attaches at the source endpoint of the parent's match, 1: destination
    int dir;      // 0: child is an out-edge of the shared vertex, 1: an in-edge
    int beta;     // -1: child precedes the parent, +1: follows it, 0: unordered (partial orders)
    int leaf;
    int copies;   // leaf children with the same side, direction and time side share
                  // one window: the factor is raised to this power (0: folded into another)
    const void* qt[2];
    const void* qn[2];
};

struct LevelArgs {
    DevGraph G;
    int64_t delta;
    int64_t ilen;   // interval unit (delta, or one interval over all times)
    int exclude;    // constraint 2: drop the run of the excluded far endpoint
    int nc;
    ChildDesc c[kMaxSlots];
    int walk;          // -1: eid order; 0 / 1: the T order of the out- / in-lists
    int4* win[kMaxSlots][2];  // per child and parity: its windows, stride 2, by walk position (null: not kept)
    void* out[2];      // per parity (interleaved, stride 2): by eid, or by T position in list out_pos_dir
    int out_pos_dir;   // first of two passes: its own walk (consecutive writes), else -1
    const void* in[2]; // second of two passes: the first pass's products ...
    int in_pos_dir;    // ... by T position in this list
    int* ovf;
    unsigned long long* nbytes;  // counting variant: access-model bytes of the launch
};

// Element i (0 or 1) of a two-entry argument array, as a select between the
// two loaded values: indexing the kernel's argument arrays at run time had
// the compiler copy all of its arguments to scratch, and so did a plain
// select, which the optimiser may turn back into a select of the two
// addresses.  The empty asm statement pins both values in scalar registers
// first (the arrays are kernel arguments: uniform across the wave).
template <typename T>
__device__ __forceinline__ T sel2(const T (&arr)[2], int i) {
    T x0 = arr[0], x1 = arr[1];
    asm("" : "+s"(x0), "+s"(x1));
    return i ? x1 : x0;
}

template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(static_cast<F&&>(f));
    }
}

// NB window bounds in a vertex's list: p[j] the first position, in T order,
// whose time is >= x_j, and q[j] the first, in N order, whose packed key is
// >= (o << bt) + x_j (three bounds for a child on one side of its parent in
// time, four for one a partial order leaves unordered).  x is clipped to
// [0, T + 1]; the key for x = T + 1 (the end of o's run) is taken as
// "> (o << bt) + T", which cannot wrap even when the id and time bits fill
// all 64.
template <int NB>
struct BoundsN {
    int32_t p[NB], q[NB];
    int32_t len;  // the list's length
};

// ---------------------------------------------------------------------------
// The level kernel's window bounds.  In T order the NB bounds are searched in
// lockstep over the child's list (NB independent loads per halving step).  In
// N order each lane's keys share its excluded neighbour, so the smallest key
// is searched over the list and the others are reached by galloping from it:
// they lie in that neighbour's run, a few entries on.  (A variant in which a
// wave walking one list staged each bound's segment in LDS after two
// wave-uniform searches was measured slower than these per-lane searches,
// which mostly hit lines their neighbours fetched.)  Every
// bound is the first position whose key is >= x (BoundsN above).
// ---------------------------------------------------------------------------

// Keys before the bound of (kx, le): z < kx, or z == kx when x > T.
__device__ __forceinline__ bool key_before(u64 z, u64 kx, bool le) { return z < kx || (le && z == kx); }

// The bound of (kx, le) in [s, b), every position before s being before it:
// doubling steps from s, then halving between the last two.
__device__ __forceinline__ int32_t key_gallop(const u64* nk, int32_t s, int32_t b, u64 kx, bool le) {
    if (s >= b || !key_before(nk[s], kx, le)) return s;
    int32_t lo = s, step = 1, hi;
    while (true) {
        hi = lo + step;
        if (hi >= b) {
            hi = b;
            break;
        }
        if (!key_before(nk[hi], kx, le)) break;
        lo = hi;
        step <<= 1;
    }
    // lo is before the bound, hi is not (or is b): the bound is in (lo, hi]
    int32_t n = hi - lo;
    while (n > 1) {
        const int32_t h = n >> 1;
        lo = key_before(nk[lo + h], kx, le) ? lo + h : lo;
        n -= h;
    }
    return lo + 1;
}

// The indices of a child's bounds in nondecreasing order of x (Kind 0: a
// child before its parent, 1: after it, 2: unordered, four bounds).
template <int Kind>
__device__ __forceinline__ constexpr int bound_rank(int k) {
    return Kind == 0 ? (k == 0 ? 1 : (k == 1 ? 0 : 2)) : (Kind == 1 ? (k == 0 ? 0 : (k == 1 ? 2 : 1))
                                                                     : (k == 0 ? 1 : (k == 1 ? 0 : (k == 2 ? 3 : 2))));
}

// The first positions in [a, b) of a T order whose time is >= x[j], for NB
// bounds in lockstep (independent loads per step).  x[j] lies in [0, T + 1],
// which the time type TT holds.  With kN, the same halving steps also find
// q, the bound of (kq, leq) in the N order over the same range: its probe
// is one more independent load per step instead of a second chain of
// dependent ones after the first.
template <typename TT, int NB, bool kN>
__device__ __forceinline__ void lockstep_lower(const TT* lt, int32_t a, int32_t b, const int64_t (&x)[NB],
                                               int32_t (&p)[NB], const u64* nk, u64 kq, bool leq, int32_t& q) {
    TT xk[NB];
    int32_t c[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        xk[j] = (TT)x[j];
        c[j] = a;
    }
    int32_t cq = a;
    int32_t n = b - a;
    while (n > 1) {
        const int32_t h = n >> 1;
        TT y[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) y[j] = lt[c[j] + h];
        u64 z = 0;
        if constexpr (kN) z = nk[cq + h];
#pragma unroll
        for (int j = 0; j < NB; ++j) c[j] = y[j] < xk[j] ? c[j] + h : c[j];
        if constexpr (kN) cq = key_before(z, kq, leq) ? cq + h : cq;
        n -= h;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) p[j] = a == b ? a : c[j] + (lt[c[j]] < xk[j] ? 1 : 0);
    if constexpr (kN) q = a == b ? a : cq + (key_before(nk[cq], kq, leq) ? 1 : 0);
}

template <int NB, int Kind>
__device__ __forceinline__ BoundsN<NB> level_bounds(const DevGraph& G, int dir, int32_t g, int32_t o,
                                                    const int64_t (&xs)[NB], bool exclude) {
    const int32_t a = sel2(G.off, dir)[g], b = sel2(G.off, dir)[g + 1];
    const u64* nk = sel2(G.nkey, dir);
    int64_t x[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) x[j] = xs[j] < 0 ? 0 : (xs[j] > G.T + 1 ? G.T + 1 : xs[j]);
    BoundsN<NB> r;
    r.len = b - a;
    const uint32_t* lt32 = sel2(G.lt32, dir);
    if (!exclude || a == b) {
        // T order only: no excluded run
        int32_t unused = a;
        if (lt32)
            lockstep_lower<uint32_t, NB, false>(lt32, a, b, x, r.p, nk, 0, false, unused);
        else
            lockstep_lower<int64_t, NB, false>(sel2(G.lt, dir), a, b, x, r.p, nk, 0, false, unused);
#pragma unroll
        for (int j = 0; j < NB; ++j) r.q[j] = a;
        return r;
    }
    // N order: all of the lane's keys share the excluded neighbour o; the
    // smallest is searched together with the T-order bounds, the others are
    // reached by galloping from it (they lie a few entries on, in o's run)
    const u64 base = (u64)o << G.bt;
    u64 kx[NB];
    bool le[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        le[j] = x[j] > G.T;
        kx[j] = base + (u64)(le[j] ? G.T : x[j]);
    }
    constexpr int j0 = bound_rank<Kind>(0);
    int32_t q0 = a;
    if (lt32)
        lockstep_lower<uint32_t, NB, true>(lt32, a, b, x, r.p, nk, kx[j0], le[j0], q0);
    else
        lockstep_lower<int64_t, NB, true>(sel2(G.lt, dir), a, b, x, r.p, nk, kx[j0], le[j0], q0);
    r.q[j0] = q0;
    sfor<1, NB>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr int jk = bound_rank<Kind>(k), jp = bound_rank<Kind>(k - 1);
        r.q[jk] = key_gallop(nk, r.q[jp], b, kx[jk], le[jk]);
    });
    return r;
}

// Sum of the child's weights over T positions [p0, p1) minus the N run [q0, q1).
template <typename W>
__device__ __forceinline__ W window_mass(int32_t p0, int32_t p1, int32_t q0, int32_t q1, bool leaf,
                                         const void* qt, const void* qn) {
    if (p1 <= p0) return (W)0;
    if (leaf) return (W)((p1 - p0) - (q1 - q0));
    const W* T = static_cast<const W*>(qt);
    const W* N = static_cast<const W*>(qn);
    return (T[p1] - T[p0]) - (N[q1] - N[q0]);
}

// One thread per edge e and both intervals holding it: slot A is
// i = floor(t / L) = blk, slot B is i - 1 (L: the interval unit).  Clipped to
// those intervals, a child window [t - delta, t] becomes
// [max(t - delta, blk L), t] (A) and [max(t - delta, (blk - 1) L), t] (B), and
// [t, t + delta] becomes [t, min(t + delta, (blk + 2) L - 1)] (A) and
// [t, min(t + delta, (blk + 1) L - 1)] (B): three distinct bounds per child
// (with L = delta: [blk delta, t], [t - delta, t], [t, t + delta] and
// [t, (blk + 1) delta - 1]).
//
// A child that a partial order leaves unordered with its parent (kPO, beta
// 0) has the window [t - delta, t + delta]: clipped, A = [max(t - delta,
// blk L), min(t + delta, (blk + 2) L - 1)] and B = [max(t - delta,
// (blk - 1) L), min(t + delta, (blk + 1) L - 1)], four distinct bounds.
//
// The counting variant returns the bytes the edge's work reads and writes
// under the access model: each read or write its element size; a list search
// of L entries ceil(log2 L) + 1 probes of each of its six bounds (three in
// the T order, of the list's time size, and three 8 B keys in the N order;
// eight bounds for an unordered child).
template <typename W, bool kCount, bool kPO>
__device__ __forceinline__ u64 level_edge(const LevelArgs& a, int64_t p) {
    const DevGraph& G = a.G;
    u64 nb = 0;
    // the walked edge: its list's owner, neighbour and time sit at p
    const int32_t e = a.walk < 0 ? (int32_t)p : sel2(G.leid, a.walk)[p];
    int32_t u, v;
    int64_t t;
    // T-order times in bytes (4 in 32-bit lists)
    const u64 tsz = G.lt32[0] ? 4 : 8;
    if constexpr (kCount) nb += a.walk < 0 ? 16 : 12 + tsz;
    if (a.walk < 0 || !sel2(G.lown, a.walk)) {
        u = G.src[e];
        v = G.dst[e];
        t = G.t[e];
    } else {
        const int32_t own = sel2(G.lown, a.walk)[p];
        int32_t nbr;
        list_entry(sel2(G.lnt, a.walk), sel2(G.lnbr, a.walk), sel2(G.lt, a.walk), p, nbr, t);
        u = a.walk == 0 ? own : nbr;
        v = a.walk == 0 ? nbr : own;
    }
    const int64_t blk = t / a.ilen;
    const bool hasB = blk >= 1;
    const int parA = (int)(blk & 1), parB = parA ^ 1;
    W prodA = 1, prodB = hasB ? (W)1 : (W)0;
    if (a.in[0]) {
        const int64_t ip = a.in_pos_dir == a.walk ? p : (int64_t)sel2(G.tpos, a.in_pos_dir)[e];
        prodA = static_cast<const W*>(sel2(a.in, parA))[2 * ip];
        prodB = hasB ? static_cast<const W*>(sel2(a.in, parB))[2 * ip] : (W)0;
        if constexpr (kCount) nb += (a.in_pos_dir == a.walk ? 0 : 4) + sizeof(W) * (hasB ? 2 : 1);
    }
    bool ovf = false;
    sfor<0, kMaxSlots>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        if (c >= a.nc) return;
        const ChildDesc& d = a.c[c];
        if (d.copies == 0) return;
        const int32_t g = d.side ? v : u;
        const int32_t o = d.side ? u : v;
        // the windows of intervals blk (parity A) and blk - 1 (B) as four
        // bounds: A = [p0, p2), B = [p1, p3) (likewise q), whatever the
        // child's side in time, so that one path below serves every child
        // (separate paths had the compiler copy the arguments to scratch)
        BoundsN<4> r;
        if (kPO && d.beta == 0) {
            const int64_t lo = t - a.delta, hi = t + a.delta;
            int64_t xs[4];
            xs[0] = lo > blk * a.ilen ? lo : blk * a.ilen;
            xs[1] = lo > (blk - 1) * a.ilen ? lo : (blk - 1) * a.ilen;
            xs[2] = (hi < (blk + 2) * a.ilen - 1 ? hi : (blk + 2) * a.ilen - 1) + 1;
            xs[3] = (hi < (blk + 1) * a.ilen - 1 ? hi : (blk + 1) * a.ilen - 1) + 1;
            r = level_bounds<4, 2>(G, d.dir, g, o, xs, a.exclude != 0);
            if constexpr (kCount) {
                int it = 0;
                for (int32_t n = r.len; n > 1; n -= n >> 1) ++it;
                nb += 8 + (4 * tsz + 32) * (u64)(it + (r.len > 0 ? 1 : 0));
            }
        } else {
            // x values (first position with time >= x):
            //   before: A = [x0, x2), B = [x1, x2) with x0 = blk delta, x1 = t - delta, x2 = t + 1
            //   after:  A = [x0, x1), B = [x0, x2) with x0 = t, x1 = t + delta + 1, x2 = (blk + 1) delta
            int64_t xs[3];
            if (d.beta < 0) {
                const int64_t lo = t - a.delta;
                xs[0] = lo > blk * a.ilen ? lo : blk * a.ilen;
                xs[1] = lo > (blk - 1) * a.ilen ? lo : (blk - 1) * a.ilen;
                xs[2] = t + 1;
            } else {
                const int64_t hi = t + a.delta;
                xs[0] = t;
                xs[1] = (hi < (blk + 2) * a.ilen - 1 ? hi : (blk + 2) * a.ilen - 1) + 1;
                xs[2] = (hi < (blk + 1) * a.ilen - 1 ? hi : (blk + 1) * a.ilen - 1) + 1;
            }
            const BoundsN<3> r3 = d.beta < 0 ? level_bounds<3, 0>(G, d.dir, g, o, xs, a.exclude != 0)
                                             : level_bounds<3, 1>(G, d.dir, g, o, xs, a.exclude != 0);
            // before: (p0, p1, p2, p2); after: (p0, p0, p1, p2)
            const bool bef = d.beta < 0;
            r.p[0] = r3.p[0];
            r.p[1] = bef ? r3.p[1] : r3.p[0];
            r.p[2] = bef ? r3.p[2] : r3.p[1];
            r.p[3] = r3.p[2];
            r.q[0] = r3.q[0];
            r.q[1] = bef ? r3.q[1] : r3.q[0];
            r.q[2] = bef ? r3.q[2] : r3.q[1];
            r.q[3] = r3.q[2];
            r.len = r3.len;
            if constexpr (kCount) {
                int it = 0;
                for (int32_t n = r.len; n > 1; n -= n >> 1) ++it;
                nb += 8 + (3 * tsz + 24) * (u64)(it + (r.len > 0 ? 1 : 0));
            }
        }
        if constexpr (kCount) {
            if (a.win[c][0]) nb += 32;
            // the prefix reads of the two windows' masses (below)
            if (!d.leaf) nb += (r.p[2] > r.p[0] ? 4 * sizeof(W) : 0) + (hasB && r.p[3] > r.p[1] ? 4 * sizeof(W) : 0);
        }
        if (a.win[c][0]) {
            // at the parent's walk position: consecutive lanes fill whole
            // lines, written past the caches so that the stream of records
            // does not evict the lines the searches reuse
            typedef int v4i __attribute__((ext_vector_type(4)));
            const v4i va = {r.p[0], r.p[2], r.q[0], r.q[2]};
            const v4i vb = hasB ? v4i{r.p[1], r.p[3], r.q[1], r.q[3]} : v4i{0, 0, 0, 0};
            __builtin_nontemporal_store(va, reinterpret_cast<v4i*>(sel2(a.win[c], parA) + 2 * p));
            __builtin_nontemporal_store(vb, reinterpret_cast<v4i*>(sel2(a.win[c], parB) + 2 * p));
        }
        const W xa = window_mass<W>(r.p[0], r.p[2], r.q[0], r.q[2], d.leaf, sel2(d.qt, parA), sel2(d.qn, parA));
        const W xb = hasB ? window_mass<W>(r.p[1], r.p[3], r.q[1], r.q[3], d.leaf, sel2(d.qt, parB), sel2(d.qn, parB)) : (W)0;
        for (int r = 0; r < d.copies; ++r) {
            if (!mul_ok(prodA, xa, &prodA)) ovf = true;
            if (!mul_ok(prodB, xb, &prodB)) ovf = true;
        }
    });
    const int64_t at = a.out_pos_dir < 0 ? (int64_t)e : (a.out_pos_dir == a.walk ? p : (int64_t)sel2(G.tpos, a.out_pos_dir)[e]);
    static_cast<W*>(sel2(a.out, parA))[2 * at] = prodA;
    static_cast<W*>(sel2(a.out, parB))[2 * at] = hasB ? prodB : (W)0;
    if constexpr (kCount) nb += 2 * sizeof(W) + (a.out_pos_dir < 0 || a.out_pos_dir == a.walk ? 0 : 4);
    if (ovf) atomicOr(a.ovf, 4);
    return nb;
}

template <typename W, bool kCount, bool kPO>
__global__ void __launch_bounds__(kBlock) level_kernel(LevelArgs a) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    u64 nb = 0;
    if (p < a.G.m) nb = level_edge<W, kCount, kPO>(a, p);
    if constexpr (kCount) {
        // one addition per workgroup
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) nb += __shfl_xor(nb, m, 64);
        __shared__ u64 part[kBlock / 64];
        if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = nb;
        __syncthreads();
        if (threadIdx.x == 0) {
            u64 sum = 0;
            for (int w = 0; w < kBlock / 64; ++w) sum += part[w];
            atomicAdd(a.nbytes, (unsigned long long)sum);
        }
    }
}

// Values of one parity held in a list's T order, read in that list's N
// order (through the N-to-T cross index, which stays inside each vertex's
// list).
// (Level values interleave their two parities, one record per position:
// both parities' scans run together and read each record once.)
template <typename W>
struct ListGather {
    const W* val;
    const int32_t* at;
    __device__ Pair2<W> operator()(int64_t p) const {
        const W* r = val + 2 * (int64_t)at[p];
        return {r[0], r[1]};
    }
};

template <typename W>
struct Plain {
    const W* val;
    __device__ Pair2<W> operator()(int64_t p) const {
        const W* r = val + 2 * p;
        return {r[0], r[1]};
    }
};

// Every 2^kCoarseBits-th entry of a prefix table.
template <typename W>
__global__ void coarse_kernel(const W* q, int64_t nc, W* c) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < nc) c[i] = q[i << kCoarseBits];
}

// Interval bounds: I_i = [i delta, (i+2) delta) holds eids [lo_i, hi_i).
__global__ void interval_kernel(const int64_t* t, int64_t m, int64_t q, int64_t delta, int32_t* lo,
                                int32_t* hi) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= q) return;
    lo[i] = lower_bound_pos<int64_t>(t, 0, (int32_t)m, i * delta);
    hi[i] = lower_bound_pos<int64_t>(t, lo[i], (int32_t)m, (i + 2) * delta);
}

// W_i = sum of w_i(c, e) over I_i: a difference of the center's prefix array.
template <typename W>
struct IntervalWeight {
    const W* qc0;
    const W* qc1;
    const int32_t* lo;
    const int32_t* hi;
    __device__ W operator()(int64_t i) const {
        const W* q = (i & 1) ? qc1 : qc0;
        return q[hi[i]] - q[lo[i]];
    }
};

// Guide entry b: the root pair of the draw X = b 2^(128 - gb) (X = 2^128 - 1
// for the last), found by the plain search; W is read from the table.
template <typename W>
__global__ void __launch_bounds__(kBlock)
guide_kernel(const W* cum, const void* qc0, const void* qc1, const int32_t* ilo, const int32_t* ihi, int64_t q,
             const int32_t* tpos0, int gb, RootGuide* guide) {
    const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t B = (int64_t)1 << gb;
    if (b > B) return;
    const W Wt = cum[q];
    if (Wt == 0) {
        guide[b].pair = 0;
        guide[b].key = 0;
        return;
    }
    X128 X;
    if (b == B) {
        X.lo = ~0ull;
        X.hi = ~0ull;
    } else {
        X.lo = 0;
        X.hi = (u64)b << (64 - gb);
    }
    const W r = scale(X, Wt);
    const void* qc[2] = {qc0, qc1};
    int32_t i = 0, e = 0;
    if (!root_pair<W>(cum, qc, ilo, ihi, q, r, 0, (int32_t)q - 1, -1, 0x7fffffff, i, e)) i = e = 0;
    guide[b].pair = ((u64)(uint32_t)i << 32) | (uint32_t)e;
    guide[b].key = (u64)((uint32_t)tpos0[e] * 2u + (uint32_t)(i & 1));
}

// The guide of gb bits in two steps: every 2^kGuideStepBits-th entry (a
// guide of gb - kGuideStepBits bits, guide_kernel), then every entry between
// two of those by the search they bound, as a root draw bounds its search by
// two guide entries (the pair is monotone in the draw).
constexpr int kGuideStepBits = 4;

template <typename W>
__global__ void __launch_bounds__(kBlock)
guide_fill_kernel(const W* cum, const void* qc0, const void* qc1, const int32_t* ilo, const int32_t* ihi,
                  const W* ioff, int64_t q, const int32_t* tpos0, int gb, const RootGuide* coarse,
                  RootGuide* guide) {
    const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t B = (int64_t)1 << gb;
    if (b > B) return;
    const int64_t c = b >> kGuideStepBits;
    // entry B (the largest draw) and the multiples of the step are coarse entries
    if ((b & ((1 << kGuideStepBits) - 1)) == 0) {
        guide[b] = coarse[c];
        return;
    }
    const RootGuide g0 = coarse[c], g1 = coarse[c + 1];
    if (g0.pair == g1.pair) {
        guide[b] = g0;
        return;
    }
    X128 X;
    X.lo = 0;
    X.hi = (u64)b << (64 - gb);
    const W r = scale(X, cum[q]);
    const void* qc[2] = {qc0, qc1};
    int32_t i = 0, e = 0;
    if (!root_pair<W>(cum, qc, ilo, ihi, q, r, (int32_t)(g0.pair >> 32), (int32_t)(g1.pair >> 32),
                      (int32_t)(uint32_t)g0.pair, (int32_t)(uint32_t)g1.pair, i, e, nullptr, ioff))
        i = e = 0;
    guide[b].pair = ((u64)(uint32_t)i << 32) | (uint32_t)e;
    guide[b].key = (u64)((uint32_t)tpos0[e] * 2u + (uint32_t)(i & 1));
}

// ioff[i] = cum[i] - qc_{i mod 2}[lo_i], modulo the word size.
template <typename W>
__global__ void __launch_bounds__(kBlock)
ioff_kernel(const W* cum, const W* qc0, const W* qc1, const int32_t* ilo, int64_t q, W* ioff) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= q) return;
    const W* qq = (i & 1) ? qc1 : qc0;
    ioff[i] = cum[i] - qq[ilo[i]];
}

unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// A prefix array read back as its values: consecutive differences modulo
// 2^64, which are the exact values whenever each value is below 2^64 (the
// level kernels flag any product that is not), however the sums wrapped.
struct WrappedDiff {
    const u64* q0;
    const u64* q1;
    __device__ Pair2<u128> operator()(int64_t p) const {
        return {(u128)(u64)(q0[p + 1] - q0[p]), (u128)(u64)(q1[p + 1] - q1[p])};
    }
};

// The center's prefix arrays in eid order from src (its values, both parities
// in one pass), then the interval bounds, the prefix of W_i, the per-interval
// offsets and the root guide.  ovf: the flag word of these scans.
template <typename W, typename R>
int finish_tables(tm_weights* w, hipStream_t st, int* ovf, const R& src) {
    tm_graph* g = w->g;
    const HostPlan& P = w->plan;
    const int64_t m = g->m;
    W* qc[2];
    for (int par = 0; par < 2; ++par) {
        TM_TRY(arena_alloc(w->arena, &qc[par], (size_t)m + 1));
        w->qc[par] = qc[par];
    }
    TM_TRY(device_exclusive_scan2<W>(src, m, qc[0], qc[1], ovf, st));
    // intervals and their weights
    TM_TRY(arena_alloc(w->arena, &w->ilo, (size_t)w->q));
    TM_TRY(arena_alloc(w->arena, &w->ihi, (size_t)w->q));
    hipLaunchKernelGGL(interval_kernel, dim3(grid_for(w->q)), dim3(kBlock), 0, st, g->d.t, m, w->q,
                       w->ilen, w->ilo, w->ihi);
    TM_HIP(hipGetLastError());
    W* cum;
    TM_TRY(arena_alloc(w->arena, &cum, (size_t)w->q + 1));
    TM_TRY(device_exclusive_scan<W>(
        IntervalWeight<W>{static_cast<const W*>(w->qc[0]), static_cast<const W*>(w->qc[1]), w->ilo,
                          w->ihi},
        w->q, cum, ovf, st));
    w->cumW = cum;
    // per-interval offsets and the root guide
    W* ioff;
    TM_TRY(arena_alloc(w->arena, &ioff, (size_t)w->q));
    hipLaunchKernelGGL((ioff_kernel<W>), dim3(grid_for(w->q)), dim3(kBlock), 0, st, (const W*)cum,
                       (const W*)w->qc[0], (const W*)w->qc[1], (const int32_t*)w->ilo, w->q, ioff);
    TM_HIP(hipGetLastError());
    w->ioff = ioff;
    w->guide_bits = guide_bits_for(m, w->lean);
    const int gc = w->guide_bits - kGuideStepBits;
    const int64_t nb = ((int64_t)1 << w->guide_bits) + 1, nc = ((int64_t)1 << gc) + 1;
    TM_TRY(arena_alloc(w->arena, &w->guide, (size_t)nb));
    RootGuide* coarse = nullptr;
    TM_HIP(dev_alloc((void**)&coarse, (size_t)nc * sizeof(RootGuide), st));
    hipLaunchKernelGGL((guide_kernel<W>), dim3(grid_for(nc)), dim3(kBlock), 0, st, (const W*)cum, w->qc[0],
                       w->qc[1], w->ilo, w->ihi, w->q, w->g->d.tpos[P.root_dir], gc, coarse);
    TM_HIP(hipGetLastError());
    hipLaunchKernelGGL((guide_fill_kernel<W>), dim3(grid_for(nb)), dim3(kBlock), 0, st, (const W*)cum,
                       w->qc[0], w->qc[1], w->ilo, w->ihi, (const W*)ioff, w->q, w->g->d.tpos[P.root_dir],
                       w->guide_bits, (const RootGuide*)coarse, w->guide);
    TM_HIP(hipGetLastError());
    TM_HIP(dev_free(coarse, st));
    return TM_OK;
}

// check_each_level: read the overflow flag after every level and stop at the
// first overflow (the synchronous build, which then restarts in 128 bits).
// ovf: the flag of the level kernels and of the non-center prefix sums;
// ovf_c: the flag of the center's prefix sums and the interval totals (the
// caller may pass ovf for both).  When only ovf_c is set, every per-edge
// value was exact and only the totals along eid order outgrew W.
template <typename W>
// nbytes (optional): the level kernels' access-model bytes are added there.
// level_timers (optional): each level launch's stage timer, for the caller to
// finish once the stream is synchronised.
int build_typed(tm_weights* w, hipStream_t st, int* ovf, int* ovf_c, bool check_each_level = false,
                unsigned long long* nbytes = nullptr,
                std::vector<std::unique_ptr<StageTimer>>* level_timers = nullptr) {
    tm_graph* g = w->g;
    const HostPlan& P = w->plan;
    const int64_t m = g->m;
    const int64_t delta = P.mo.delta;
    w->has_win = !w->lean && weights_keep_windows(P, m);
    // bottom-up over heights; leaves other than the center have weight 1 and
    // no table (a lone center edge gets a table of ones)
    for (int h = 0; h <= P.H; ++h) {
        for (int s = 0; s < P.nt; ++s) {
            if (P.height[s] != h || (h == 0 && s != 0)) continue;
            // children grouped by the endpoint they attach at: each group
            // walks the lists of that endpoint, so neighbouring lanes search
            // the same list at nearby times; with children at both endpoints
            // the first pass leaves its products where the second walks
            std::vector<int> grp[2];
            for (int j = 0; j < P.n_children[s]; ++j) grp[P.side[P.children[s][j]]].push_back(P.children[s][j]);
            const bool two = !grp[0].empty() && !grp[1].empty();
            // both parities of an edge in one record: parity par of position
            // x at [2 x + par], so a scattered write touches one line
            {
                W* p;
                TM_HIP(dev_alloc((void**)&p, ((size_t)2 * m * sizeof(W) + 255) & ~(size_t)255, st));
                w->vals[s][0] = p;
            }
            W* tmp = nullptr;
            if (two) TM_HIP(dev_alloc((void**)&tmp, ((size_t)2 * m * sizeof(W) + 255) & ~(size_t)255, st));
            int prev_walk = -1;
            for (int pass = 0; pass < (two ? 2 : 1); ++pass) {
                const int side = two ? pass : (grp[0].empty() ? 1 : 0);
                const std::vector<int>& cs = grp[side];
                LevelArgs a;
                std::memset(&a, 0, sizeof a);
                a.G = g->d;
                a.delta = delta;
                a.ilen = w->ilen;
                a.exclude = (w->constraints & TM_C_EXCLUDE) ? 1 : 0;
                a.nc = (int)cs.size();
                for (int j = 0; j < a.nc; ++j) {
                    const int c = cs[j];
                    ChildDesc& d = a.c[j];
                    d.side = P.side[c];
                    d.dir = P.alpha[c] > 0 ? 0 : 1;
                    d.beta = P.beta[c];
                    d.leaf = P.n_children[c] == 0;
                    d.copies = 1;
                    for (int j2 = 0; j2 < j && d.leaf; ++j2) {
                        ChildDesc& e2 = a.c[j2];
                        if (e2.leaf && e2.copies > 0 && e2.dir == d.dir && e2.beta == d.beta) {
                            ++e2.copies;
                            d.copies = 0;
                            break;
                        }
                    }
                    for (int par = 0; par < 2; ++par) {
                        d.qt[par] = w->qt[c][par];
                        d.qn[par] = w->qn[c][par];
                    }
                }
                if (w->has_win) {
                    // a folded leaf shares the window of the child it joins
                    for (int j = 0; j < a.nc; ++j) {
                        const int c = cs[j];
                        if (a.c[j].copies > 0) {
                            // both parities of an edge in one 32-byte record
                            TM_TRY(arena_alloc(w->arena, &w->win[c][0], 2 * (size_t)m));
                            w->win[c][1] = w->win[c][0] + 1;
                            for (int par = 0; par < 2; ++par) a.win[j][par] = w->win[c][par];
                        } else {
                            for (int j2 = 0; j2 < j; ++j2) {
                                const ChildDesc& e2 = a.c[j2];
                                if (e2.leaf && e2.copies > 0 && e2.dir == a.c[j].dir && e2.beta == a.c[j].beta) {
                                    for (int par = 0; par < 2; ++par) w->win[c][par] = w->win[cs[j2]][par];
                                    break;
                                }
                            }
                        }
                    }
                }
                // each pass walks the list its children attach to, so that
                // neighbouring lanes search one list (the center's root list
                // is that list too when all its children attach at one end);
                // the kept windows are written in that walk order, and the
                // sampler finds a parent's walk position through tpos when it
                // drew the parent from the other list
                a.walk = a.nc == 0 ? -1 : side;
                for (int par = 0; par < 2; ++par) {
                    a.out[par] = ((two && pass == 0) ? tmp : static_cast<W*>(w->vals[s][0])) + par;
                    a.in[par] = (two && pass == 1) ? (const void*)(tmp + par) : nullptr;
                }
                // the first of two passes leaves its products in its own walk
                // order; the second gathers them
                // a non-center slot's values land at its T-order position in
                // the list its parent searches (that list's prefix arrays
                // then scan them in place); the center's in eid order
                const int own_dir = s == 0 ? -1 : (P.alpha[s] > 0 ? 0 : 1);
                a.out_pos_dir = (two && pass == 0) ? a.walk : own_dir;
                a.in_pos_dir = prev_walk;
                prev_walk = a.walk;
                a.ovf = ovf;
                a.nbytes = nbytes;
                StageTimer* lt = nullptr;
                if (level_timers) {
                    level_timers->push_back(std::make_unique<StageTimer>());
                    lt = level_timers->back().get();
                    lt->start(TM_STAGE_LEVELS, st);
                }
                // children a partial order leaves unordered take the
                // four-bound form, compiled only into its own variant
                bool unordered = false;
                for (int j = 0; j < a.nc; ++j) unordered = unordered || a.c[j].beta == 0;
                if (unordered) {
                    if (nbytes)
                        hipLaunchKernelGGL((level_kernel<W, true, true>), dim3(grid_for(m)), dim3(kBlock), 0, st, a);
                    else
                        hipLaunchKernelGGL((level_kernel<W, false, true>), dim3(grid_for(m)), dim3(kBlock), 0, st, a);
                } else if (nbytes) {
                    hipLaunchKernelGGL((level_kernel<W, true, false>), dim3(grid_for(m)), dim3(kBlock), 0, st, a);
                } else {
                    hipLaunchKernelGGL((level_kernel<W, false, false>), dim3(grid_for(m)), dim3(kBlock), 0, st, a);
                }
                TM_HIP(hipGetLastError());
                if (lt) lt->stop();
            }
            if (two) TM_HIP(dev_free(tmp, st));
            if (check_each_level && sizeof(W) == 8) {
                int h_ovf = 0;
                TM_HIP(hipMemcpyAsync(&h_ovf, ovf, sizeof(int), hipMemcpyDeviceToHost, st));
                TM_HIP(sync_stream(st));
                if (h_ovf) return TM_OK;  // the caller sees the flag and widens
            }
            // prefix sums along the lists the parent searches
            if (s != 0) {
                const int dir = P.alpha[s] > 0 ? 0 : 1;
                W *qt[2], *qn[2];
                for (int par = 0; par < 2; ++par) {
                    TM_TRY(arena_alloc(w->arena, &qt[par], (size_t)m + 1));
                    TM_TRY(arena_alloc(w->arena, &qn[par], (size_t)m + 1));
                    w->qt[s][par] = qt[par];
                    w->qn[s][par] = qn[par];
                }
                const W* vp = static_cast<const W*>(w->vals[s][0]);
                TM_TRY(device_exclusive_scan2<W>(Plain<W>{vp}, m, qt[0], qt[1], ovf, st));
                TM_TRY(device_exclusive_scan2<W>(ListGather<W>{vp, g->d.nxref[dir]}, m, qn[0], qn[1], ovf, st));
                // lean sets (memory over speed) search the full tables
                const int64_t nc = (m >> kCoarseBits) + 1;
                for (int par = 0; par < 2 && !w->lean; ++par) {
                    W* c;
                    TM_TRY(arena_alloc(w->arena, &c, (size_t)nc));
                    hipLaunchKernelGGL((coarse_kernel<W>), dim3(grid_for(nc)), dim3(kBlock), 0, st,
                                       (const W*)qt[par], nc, c);
                    TM_HIP(hipGetLastError());
                    w->qtc[s][par] = c;
                }
                TM_HIP(dev_free(w->vals[s][0], st));
                w->vals[s][0] = nullptr;
            }
        }
    }
    // the center: prefix sums in eid order (slot 0 is the center), then the
    // interval tables
    {
        TM_TRY(finish_tables<W>(w, st, ovf_c, Plain<W>{static_cast<const W*>(w->vals[0][0])}));
    }
    TM_HIP(dev_free(w->vals[0][0], st));
    w->vals[0][0] = nullptr;
    return TM_OK;
}

// The 64-bit tables made 128-bit without recomputing any level: every
// per-edge value is exact (no product overflowed) and only the center's
// totals along eid order outgrew 64 bits.  The list tables stay as they are
// (exact in 64 bits; readers widen their entries); the center's prefix
// arrays are rebuilt in 128 bits from their own consecutive differences, and
// the interval tables and the guide follow.  Kept windows are positions and
// stay.
int widen_tables(tm_weights* w, hipStream_t st, int* ovf) {
    const int64_t m = w->g->m;
    const size_t old_bytes = (size_t)(m + 1) * sizeof(u64);
    const void* qc64[2] = {w->qc[0], w->qc[1]};
    void* old[6] = {w->qc[0], w->qc[1], w->ilo, w->ihi, w->cumW, w->ioff};
    const size_t old_sz[6] = {old_bytes, old_bytes, (size_t)w->q * 4, (size_t)w->q * 4,
                              (size_t)(w->q + 1) * 8, (size_t)w->q * 8};
    void* old_guide = w->guide;
    const size_t guide_sz = (((size_t)1 << w->guide_bits) + 1) * sizeof(RootGuide);
    const WrappedDiff src{static_cast<const u64*>(qc64[0]), static_cast<const u64*>(qc64[1])};
    w->wide = true;
    TM_TRY(finish_tables<u128>(w, st, ovf, src));
    for (int x = 0; x < 6; ++x) w->arena.release_one(old[x], old_sz[x]);
    w->arena.release_one(old_guide, guide_sz);
    return TM_OK;
}

void clear_tables(tm_weights* w) {
    w->arena.release();
    for (auto& vs : w->vals)
        for (void* v : vs)
            if (v) (void)dev_free(v, w->arena.stream);
    std::memset(w->vals, 0, sizeof w->vals);
    std::memset(w->win, 0, sizeof w->win);
    w->has_win = false;
    std::memset(w->qt, 0, sizeof w->qt);
    std::memset(w->qn, 0, sizeof w->qn);
    std::memset(w->qtc, 0, sizeof w->qtc);
    std::memset(w->qc, 0, sizeof w->qc);
    w->ilo = w->ihi = nullptr;
    w->cumW = nullptr;
    w->guide = nullptr;
    w->ioff = nullptr;
}

}  // namespace

int64_t interval_unit(const tm_weights* w) {
    return (w->constraints & TM_C_WINDOWS) ? w->plan.mo.delta : w->g->T + 1;
}

int weights_build(tm_weights* w, hipStream_t st, u64* model_bytes) {
    tm_graph* g = w->g;
    w->ilen = interval_unit(w);
    w->q = g->m > 0 ? g->T / w->ilen + 1 : 0;
    if (g->m == 0) {
        w->W = 0;
        w->wide = false;
        w->list_wide = false;
        return TM_OK;
    }
    if (w->q >= ((int64_t)1 << 31)) return tm_fail(TM_ERANGE, "weights: too many intervals");
    StageTimer timer;
    timer.start(TM_STAGE_WEIGHTS, st);
    std::vector<std::unique_ptr<StageTimer>> level_timers;
    int* ovf = nullptr;
    TM_HIP(dev_alloc((void**)&ovf, 2 * sizeof(int), st));
    // the level kernels' access-model bytes, over every attempt
    unsigned long long* nbytes = nullptr;
    u64 hbytes = 0;
    if (model_bytes) {
        TM_HIP(dev_alloc((void**)&nbytes, sizeof(u64), st));
        TM_TRY(fill_u32(nbytes, 2, 0u, st));
    }
    int h = 0;
    int rc = TM_OK;
    // ovf + 1: the 64-bit build's center and interval totals (see build_typed)
    int* ovf_c = ovf + 1;
    w->needs_wide = false;
    for (int wide = w->width_mode == 2 ? 1 : 0; wide < (w->width_mode == 1 ? 1 : 2); ++wide) {
        clear_tables(w);
        TM_TRY(fill_u32(ovf, 2, 0u, st));
        w->wide = wide != 0;
        w->list_wide = w->wide;
        // on large graphs a level costs far more than a host round trip, and
        // a server's builder thread waits alone: there the 64-bit build
        // checks after every level and stops at the first overflow; other
        // builds of small graphs check once, at the end
        const bool per_level = w->lean || g->m >= ((int64_t)1 << 23);
        rc = wide ? build_typed<u128>(w, st, ovf, ovf, false, nbytes, &level_timers)
                  : build_typed<u64>(w, st, ovf, ovf_c, per_level, nbytes, &level_timers);
        if (rc != TM_OK) break;
        int hc = 0;
        if (!wide) {
            // only totals along eid order outgrew 64 bits (no product, no
            // other list's total): widen the tables instead of rebuilding
            TM_HIP(read_back({{&h, ovf, sizeof(int)}, {&hc, ovf_c, sizeof(int)}}, st));
            if ((h != 0 || hc != 0) && w->width_mode == 1) {
                // 64 bits only: the caller decides where the 128-bit set goes
                w->needs_wide = true;
                rc = tm_fail(TM_EOVERFLOW, "weights: the set needs 128 bits");
                break;
            }
            if (h == 0 && hc != 0 && !(hc & 1) && w->cumW) {
                rc = widen_tables(w, st, ovf);
                if (rc != TM_OK) break;
            }
        }
        u64 hW[2] = {0, 0};
        timer.stop();
        // a 64-bit build that stopped at an overflowing level has no W yet
        const bool w128 = w->wide;
        const size_t wsz = w->cumW ? (w128 ? 16 : 8) : 0;
        TM_HIP(read_back({{&h, ovf, sizeof(int)},
                          {hW, static_cast<const unsigned char*>(w->cumW) + w->q * (w128 ? 16 : 8), wsz},
                          {&hbytes, nbytes, nbytes ? sizeof(u64) : 0}},
                         st));
        w->W = ((u128)hW[1] << 64) | hW[0];
        if (w128 && !wide) {
            // widened: the 128-bit totals are exact unless they wrapped 2^128
            if (h != 0) rc = tm_fail(TM_EOVERFLOW, "weights: a weight or W reaches 2^128");
            break;
        }
        if (h == 0 && hc == 0) break;
        if (wide) rc = tm_fail(TM_EOVERFLOW, "weights: a weight or W reaches 2^128");
    }
    TM_HIP(dev_free(ovf, st));
    if (nbytes) TM_HIP(dev_free(nbytes, st));
    timer.finish();
    for (auto& t : level_timers) t->finish();
    if (model_bytes) *model_bytes = hbytes;
    if (rc != TM_OK) clear_tables(w);
    return rc;
}

u64 weights_footprint(const HostPlan& P, int64_t m, int64_t q, bool wide, bool lean) {
    if (m <= 0) return 0;
    const u64 wsz = wide ? 16 : 8;
    auto blk = [](u64 bytes) { return ((bytes ? bytes : 16) + 255) & ~(u64)255; };
    u64 b = 0;
    for (int s = 1; s < P.nt; ++s)
        if (P.n_children[s] > 0)
            b += 4 * blk((u64)(m + 1) * wsz) +
                 (lean ? 0 : 2 * blk((u64)((m >> kCoarseBits) + 1) * wsz));  // qt, qn, coarse qt
    b += 2 * blk((u64)(m + 1) * wsz);                   // qc, per parity
    b += 2 * blk((u64)q * 4) + blk((u64)(q + 1) * wsz); // ilo, ihi, cumW
    b += blk((u64)q * wsz);                              // ioff
    b += blk((((u64)1 << guide_bits_for(m, lean)) + 1) * sizeof(RootGuide));  // root guide
    if (!lean && weights_keep_windows(P, m)) b += weights_window_bytes(P, m);
    return b;
}

// Child window tables of a plan: one per child that the level kernel does
// not fold into an earlier leaf sibling (same side, direction and time side).
static int window_tables(const HostPlan& P) {
    int n = 0;
    for (int s = 0; s < P.nt; ++s) {
        for (int j = 0; j < P.n_children[s]; ++j) {
            const int c = P.children[s][j];
            bool folded = false;
            for (int j2 = 0; j2 < j && P.n_children[c] == 0; ++j2) {
                const int c2 = P.children[s][j2];
                if (P.n_children[c2] == 0 && P.side[c2] == P.side[c] && P.alpha[c2] == P.alpha[c] &&
                    P.beta[c2] == P.beta[c]) {
                    folded = true;
                    break;
                }
            }
            if (!folded) ++n;
        }
    }
    return n;
}

u64 weights_window_bytes(const HostPlan& P, int64_t m) {
    if (m <= 0) return 0;
    const u64 per = (((u64)m * 2 * sizeof(int4)) + 255) & ~(u64)255;
    return (u64)window_tables(P) * per;
}

bool weights_keep_windows(const HostPlan& P, int64_t m) {
    return m > 0 && weights_window_bytes(P, m) <= kWinMaxBytes;
}

int guide_bits_for(int64_t m, bool lean) {
    int b = 0;
    while (b < 62 && ((int64_t)1 << (b + 1)) <= m) ++b;  // floor(log2 m): ~2m pairs, ~2 per bucket
    if (lean) {
        b -= 2;
        return b < 8 ? 8 : (b > 23 ? 23 : b);
    }
    b += kGuideExtraBits;
    // up to 2^26 buckets (1 GiB): at 1e8 edges 2^26 rather than 2^23 cut the
    // root draws by a third for 1.2 ms more guide build per weight set
    return b < 8 ? 8 : (b > 26 ? 26 : b);
}

u64 weights_build_extra(int64_t m, bool wide) {
    // one slot's values and a two-pass level's products, per parity; the
    // coarse root guide
    if (m <= 0) return 0;
    const u64 coarse = (((u64)1 << (guide_bits_for(m) - kGuideStepBits)) + 1) * sizeof(RootGuide);
    return 4 * ((((u64)m * (wide ? 16 : 8)) + 255) & ~(u64)255) + ((coarse + 255) & ~(u64)255);
}

int weights_enqueue(tm_weights* w, hipStream_t st, int* ovf,
                    std::vector<std::unique_ptr<StageTimer>>* level_timers) {
    tm_graph* g = w->g;
    w->ilen = interval_unit(w);
    w->q = g->m > 0 ? g->T / w->ilen + 1 : 0;
    w->wide = false;
    w->list_wide = false;
    w->W = 0;
    if (g->m == 0) return TM_OK;
    if (w->q >= ((int64_t)1 << 31)) return tm_fail(TM_ERANGE, "weights: too many intervals");
    clear_tables(w);
    const int rc = build_typed<u64>(w, st, ovf, ovf, false, nullptr, level_timers);
    if (rc != TM_OK) clear_tables(w);
    return rc;
}
