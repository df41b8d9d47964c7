// Shared definitions of the TIMEST GPU library: plain structs handed to the
// kernels, exact-integer helpers, the Philox4x32-10 generator and searches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef unsigned __int128 u128;
typedef unsigned long long u64;

#define TM_HD __host__ __device__ __forceinline__

// Block shape used by every kernel: 256 lanes = 4 wave64.
constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

// ---------------------------------------------------------------------------
// Graph in device memory.  Edges are indexed by eid (rank under (t, src, dst)).
// Per vertex g, out-lists occupy positions [out_off[g], out_off[g+1]) of two
// arrays: the T order (time, then destination: eid order restricted to g) and
// the N order (destination, then time), which holds El_{g,v} as a contiguous
// run.  In-lists likewise with the source as neighbour.  N-order entries carry
// a packed key (neighbour << bt | time) and the position of the same edge in
// the T order (xref).
// ---------------------------------------------------------------------------
struct DevGraph {
    int64_t m;
    int32_t n;
    int32_t bt;          // bits of the time field in the packed key
    int64_t T;           // largest shifted time
    const int32_t* src;  // [m]
    const int32_t* dst;  // [m]
    const int64_t* t;    // [m]
    const int32_t* off[2];     // [2][n+1]: 0 = out, 1 = in
    const int64_t* lt[2];      // T order: time (null when lt32 holds it)
    const uint32_t* lt32[2];   // T order: time in 32 bits, when every shifted time is below
                               // 2^32 - 1 (then x + 1 of any time x fits too); else null
    const int32_t* leid[2];    // T order: eid
    const int32_t* lnbr[2];    // T order: neighbour (null when lnt holds it)
    const uint2* lnt[2];       // T order, with 32-bit times: (neighbour, time) per position, one
                               // read for both (lt32 keeps the times for searches); else null
    const int32_t* lown[2];    // T order: the list's owner (source for out-lists); null
                               // above 2^28 edges (memory goes to weight sets there)
    const u64* nkey[2];        // N order: neighbour << bt | time
    const int32_t* nxref[2];   // N order: position of the edge in the T order
    const int32_t* neid[2];    // N order: eid
    const int32_t* tpos[2];    // by eid: the edge's position in the T order
};

// ---------------------------------------------------------------------------
// Exact integers.
// ---------------------------------------------------------------------------
TM_HD bool add_ok(u64 a, u64 b, u64* r) { *r = a + b; return *r >= a; }
TM_HD bool add_ok(u128 a, u128 b, u128* r) { *r = a + b; return *r >= a; }
TM_HD bool mul_ok(u64 a, u64 b, u64* r) { return !__builtin_mul_overflow(a, b, r); }
TM_HD bool mul_ok(u128 a, u128 b, u128* r) { return !__builtin_mul_overflow(a, b, r); }

template <typename T>
TM_HD u128 to_u128(T x) { return (u128)x; }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds, each multiplying words 0
// and 2 by the two round multipliers and mixing the high halves with the other
// words and the key; the key advances by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct Block4 {
    uint32_t x[4];
};

__device__ __forceinline__ Block4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                           uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Block4 b;
    b.x[0] = c0;
    b.x[1] = c1;
    b.x[2] = c2;
    b.x[3] = c3;
    return b;
}

// 128-bit block of draw d of sample j: words x0 + x1 2^32 + x2 2^64 + x3 2^96.
struct X128 {
    u64 lo, hi;
};

// Root guide entry: the root pair (interval << 32 | eid) of one evenly spaced
// draw, and that pair's sort key (T-order position of the edge in the root
// list * 2 + interval parity).  A bucket whose two ends hold the same pair
// holds only that pair.
struct alignas(16) RootGuide {
    u64 pair;
    u64 key;
};

__device__ __forceinline__ X128 draw_block(u64 seed, u64 j, uint32_t d) {
    Block4 b = philox10((uint32_t)j, (uint32_t)(j >> 32), d, 0u, (uint32_t)seed,
                        (uint32_t)(seed >> 32));
    X128 x;
    x.lo = (u64)b.x[0] | ((u64)b.x[1] << 32);
    x.hi = (u64)b.x[2] | ((u64)b.x[3] << 32);
    return x;
}

// floor(X * n / 2^128): the position selected among n.
__device__ __forceinline__ u64 scale(X128 X, u64 n) {
    // X * n = hi*n * 2^64 + lo*n; the floor by 2^128 is the top word of
    // hi*n + floor(lo*n / 2^64), which cannot carry past 128 bits.
    u128 s = (u128)X.hi * n + (u128)__umul64hi(X.lo, n);
    return (u64)(s >> 64);
}

__device__ __forceinline__ u128 scale(X128 X, u128 n) {
    const u64 n0 = (u64)n, n1 = (u64)(n >> 64);
    const u128 a = (u128)X.lo * n0;   // 2^0
    const u128 b = (u128)X.lo * n1;   // 2^64
    const u128 c = (u128)X.hi * n0;   // 2^64
    const u128 d = (u128)X.hi * n1;   // 2^128
    const u128 mid = (a >> 64) + (u64)b + (u64)c;
    return d + (b >> 64) + (c >> 64) + (mid >> 64);
}

// First index in [lo, hi) with a[idx] > key (hi if none); a fixed number of
// halving steps with no branch on the data.
template <typename T>
__device__ __forceinline__ int32_t upper_bound_bl(const T* a, int32_t lo, int32_t hi, T key) {
    int32_t n = hi - lo;
    if (n <= 0) return lo;
    int32_t b = lo;
    while (n > 1) {
        const int32_t h = n >> 1;
        b = a[b + h] <= key ? b + h : b;
        n -= h;
    }
    return b + (a[b] <= key ? 1 : 0);
}

// A list prefix table read as W: its entries are W, or 64-bit under W = u128
// when the set was widened after a 64-bit build (every entry then fits).
template <typename W>
struct ListTab {
    const void* p;
    bool wide;
    const void* c = nullptr;  // every 2^cb-th entry (same width), or null
    int cb = 0;
    __device__ __forceinline__ W operator[](int64_t i) const {
        if constexpr (sizeof(W) == 8) {
            return static_cast<const W*>(p)[i];
        } else {
            return wide ? static_cast<const u128*>(p)[i] : (u128) static_cast<const u64*>(p)[i];
        }
    }
    __device__ __forceinline__ int bytes() const { return sizeof(W) == 8 || wide ? (int)sizeof(W) : 8; }
    // upper_bound through the coarse entries: the first coarse entry above
    // key inside the range bounds the position to the 2^cb entries before
    // it, which a search of one or two lines finishes.
    __device__ __forceinline__ int32_t upper_bound_coarse(int32_t lo, int32_t hi, W key) const {
        const int32_t cl = (lo + (1 << cb) - 1) >> cb, ch = hi > 0 ? (hi - 1) >> cb : -1;
        int32_t flo = lo, fhi = hi;
        if (c && cl <= ch) {
            const ListTab<W> ct{c, wide};
            int32_t j = cl, len = ch - cl + 1;  // first coarse index in [cl, ch] above key (ch + 1 if none)
            while (len > 0) {
                const int32_t h = len >> 1;
                if (ct[j + h] <= key) {
                    j += h + 1;
                    len -= h + 1;
                } else {
                    len = h;
                }
            }
            if (j > cl) flo = ((j - 1) << cb) + 1;  // entry (j - 1) 2^cb is <= key
            if (j <= ch) fhi = (j << cb) + 1;       // entry j 2^cb is > key
        }
        int32_t a = flo, b = fhi;
        while (a < b) {
            const int32_t mid = a + ((b - a) >> 1);
            if ((*this)[mid] > key) b = mid;
            else a = mid + 1;
        }
        return a;
    }
    // the first position in [lo, hi) whose entry is > key (hi if none)
    __device__ __forceinline__ int32_t upper_bound(int32_t lo, int32_t hi, W key) const {
        if constexpr (sizeof(W) == 8) {
            return upper_bound_bl<W>(static_cast<const W*>(p), lo, hi, key);
        } else {
            if (wide) return upper_bound_bl<u128>(static_cast<const u128*>(p), lo, hi, key);
            // the entries are below 2^64: a larger key lies past all of them
            if (key >> 64) return hi;
            return upper_bound_bl<u64>(static_cast<const u64*>(p), lo, hi, (u64)key);
        }
    }
};

// The root pair drawn by r in [0, W): over pairs (interval i, eid e in I_i)
// in (i, eid) order weighted w_i(center, e), the pair whose cumulative range
// holds r -- the last interval i with cum[i] <= r, then the last e of I_i
// with qc[e] - qc[lo_i] <= r - cum[i] (qc: the center's prefix of the
// interval's parity).  The search looks only at intervals [i0, i1], at eids
// >= ea in i0 and <= eb in i1 (the range of a guide bucket; full ranges give
// the plain search).  False on tables that cannot hold r.
//
// ioff (optional): per interval, cum[i] - qc[lo_i] (mod 2^bits).  With a
// guide range inside one interval (i0 == i1, lo_i <= ea <= eb < hi_i), the
// pair is found from ioff[i0] and the eids [ea, eb] alone: r - ioff[i] is
// the target of the eid search, and the range already lies in the interval.
template <typename W>
__device__ __forceinline__ bool root_pair(const W* cum, const void* const* qc, const int32_t* ilo,
                                          const int32_t* ihi, int64_t q, W r, int32_t i0, int32_t i1,
                                          int32_t ea, int32_t eb, int32_t& i_out, int32_t& e_out,
                                          int32_t* span = nullptr, const W* ioff = nullptr) {
    if (ioff && i0 == i1 && i0 >= 0 && i0 < q && ea >= 0 && eb >= ea) {
        const W* qq = static_cast<const W*>(qc[i0 & 1]);
        const W target = r - ioff[i0];
        int32_t e = upper_bound_bl<W>(qq, ea + 1, eb + 2, target) - 1;
        e = e < ea ? ea : (e > eb ? eb : e);
        i_out = i0;
        e_out = e;
        if (span) *span = eb - ea + 1;
        return true;
    }
    const int32_t i = upper_bound_bl<W>(cum, i0, i1 + 1, r) - 1;
    if (i < 0 || i >= q) return false;
    const int32_t lo = ilo[i], hi = ihi[i];
    if (hi <= lo) return false;
    const W* qq = static_cast<const W*>(qc[i & 1]);
    const W target = r - cum[i] + qq[lo];
    int32_t slo = lo, shi = hi;
    if (i == i0 && ea > slo) slo = ea;
    if (i == i1 && eb + 1 < shi) shi = eb + 1;
    if (shi <= slo) {
        slo = lo;
        shi = hi;
    }
    int32_t e = upper_bound_bl<W>(qq, slo + 1, shi + 1, target) - 1;
    e = e < lo ? lo : (e >= hi ? hi - 1 : e);
    i_out = i;
    e_out = e;
    if (span) *span = shi - slo;
    return true;
}

// ---------------------------------------------------------------------------
// Searches over sorted ranges [lo, hi) of positions (int32 positions).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ int32_t lower_bound_pos(const T* a, int32_t lo, int32_t hi, T key) {
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// The neighbour and time at position i of a T order, given that list's
// tables: one (neighbour, time) record when the graph has 32-bit times, else
// the neighbour and 64-bit time arrays.
__device__ __forceinline__ void list_entry(const uint2* nt, const int32_t* nbr, const int64_t* lt, int64_t i,
                                           int32_t& v, int64_t& t) {
    if (nt) {
        const uint2 x = nt[i];
        v = (int32_t)x.x;
        t = (int64_t)x.y;
    } else {
        v = nbr[i];
        t = lt[i];
    }
}

template <typename T>
__device__ __forceinline__ int32_t upper_bound_pos(const T* a, int32_t lo, int32_t hi, T key) {
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (key < a[mid]) hi = mid; else lo = mid + 1;
    }
    return lo;
}

