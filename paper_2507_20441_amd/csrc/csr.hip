// Graph build: validation, the canonical edge order and the per-vertex lists.
//
// The paper stores the graph as per-vertex in/out edge lists sorted by time,
// searched by binary search (Sec. 4, storage paragraph), with timestamps
// shifted to start at 0.  Here every list is built by stable LSD radix sorts
// so that the order inside each list is the canonical eid order; each sort
// carries the edge fields its lists need (time, eid, neighbour), so the list
// arrays come out of the sorts in order and only the two inverse
// permutations (an edge's T position) are written or read at random.
#include <algorithm>
#include <cstdio>
#include <cstring>

#include "tm_primitives.h"

namespace {

enum : int { kBadRange = 1, kSelfLoop = 2, kDup = 4 };

__device__ __forceinline__ u64 order_key(int64_t t) { return (u64)t ^ 0x8000000000000000ull; }

// Per workgroup: flags and the time range of its edges, as one partial each
// (part[3 b] = min, part[3 b + 1] = max, part[3 b + 2] = flags).
__global__ void __launch_bounds__(kBlock)
validate_kernel(const int32_t* src, const int32_t* dst, const int64_t* t, int64_t m, int32_t n, u64* part) {
    u64 lo = ~0ull, hi = 0;
    int f = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * kBlock) {
        const int32_t u = src[i], v = dst[i];
        if (u < 0 || u >= n || v < 0 || v >= n) f |= kBadRange;
        if (u == v) f |= kSelfLoop;
        const u64 k = order_key(t[i]);
        lo = k < lo ? k : lo;
        hi = k > hi ? k : hi;
    }
    for (int d = 32; d > 0; d >>= 1) {
        const u64 a = __shfl_xor(lo, d, 64), b = __shfl_xor(hi, d, 64);
        lo = a < lo ? a : lo;
        hi = b > hi ? b : hi;
        f |= __shfl_xor(f, d, 64);
    }
    // one partial per block: the waves meet in LDS first
    __shared__ u64 slo[kWaves], shi[kWaves];
    __shared__ int sf[kWaves];
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        slo[wave] = lo;
        shi[wave] = hi;
        sf[wave] = f;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kWaves; ++w) {
            lo = slo[w] < lo ? slo[w] : lo;
            hi = shi[w] > hi ? shi[w] : hi;
            f |= sf[w];
        }
        part[3 * blockIdx.x] = lo;
        part[3 * blockIdx.x + 1] = hi;
        part[3 * blockIdx.x + 2] = (u64)(uint32_t)f;
    }
}

// One workgroup: the partials of nb workgroups into *flags, *tmin, *tmax.
__global__ void __launch_bounds__(kBlock)
validate_reduce_kernel(const u64* part, int nb, int* flags, u64* tmin, u64* tmax) {
    u64 lo = ~0ull, hi = 0;
    uint32_t f = 0;
    for (int b = threadIdx.x; b < nb; b += kBlock) {
        lo = part[3 * b] < lo ? part[3 * b] : lo;
        hi = part[3 * b + 1] > hi ? part[3 * b + 1] : hi;
        f |= (uint32_t)part[3 * b + 2];
    }
    for (int d = 32; d > 0; d >>= 1) {
        const u64 a = __shfl_xor(lo, d, 64), c = __shfl_xor(hi, d, 64);
        lo = a < lo ? a : lo;
        hi = c > hi ? c : hi;
        f |= (uint32_t)__shfl_xor((int)f, d, 64);
    }
    __shared__ u64 slo[kWaves], shi[kWaves];
    __shared__ uint32_t sf[kWaves];
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        slo[wave] = lo;
        shi[wave] = hi;
        sf[wave] = f;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kWaves; ++w) {
            lo = slo[w] < lo ? slo[w] : lo;
            hi = shi[w] > hi ? shi[w] : hi;
            f |= sf[w];
        }
        *tmin = lo;
        *tmax = hi;
        *flags = (int)f;
    }
}

// Sort keys for the canonical order (t, u, v): one packed key t << 2bn |
// u << bn | v when it fits 64 bits, else the key u << bn | v with the time
// carried beside it (a second sort then orders by time).
__global__ void canon_keys_kernel(const int32_t* src, const int32_t* dst, const int64_t* t, int64_t m, int64_t tmin,
                                  int bn, int one_key, u64* keys, u64* times) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= m) return;
    u64 k = ((u64)(uint32_t)src[i] << bn) | (u64)(uint32_t)dst[i];
    if (one_key)
        k |= (u64)(t[i] - tmin) << (2 * bn);
    else
        times[i] = (u64)(t[i] - tmin);
    keys[i] = k;
}

// Edge arrays from the sorted packed keys, and the duplicate check on
// neighbours.
// (ot32, when not null: the times again in 32 bits, for the list sorts)
__global__ void decode_packed_kernel(const u64* key, int64_t m, int bn, int32_t* osrc, int32_t* odst, int64_t* ot,
                                     uint32_t* ot32, int* flags) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= m) return;
    const u64 k = key[e];
    const u64 mask = (1ull << bn) - 1;
    osrc[e] = (int32_t)((k >> bn) & mask);
    odst[e] = (int32_t)(k & mask);
    ot[e] = (int64_t)(k >> (2 * bn));
    if (ot32) ot32[e] = (uint32_t)(k >> (2 * bn));
    if (e > 0 && key[e - 1] == k) atomicOr(flags, kDup);
}

// Edge arrays from the sorted times and the (u, v) keys carried with them.
__global__ void decode_split_kernel(const u64* tsorted, const u64* uv, int64_t m, int bn, int32_t* osrc,
                                    int32_t* odst, int64_t* ot, uint32_t* ot32, int* flags) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= m) return;
    const u64 k = uv[e], t = tsorted[e];
    const u64 mask = (1ull << bn) - 1;
    osrc[e] = (int32_t)(k >> bn);
    odst[e] = (int32_t)(k & mask);
    ot[e] = (int64_t)t;
    if (ot32) ot32[e] = (uint32_t)t;
    if (e > 0 && uv[e - 1] == k && tsorted[e - 1] == t) atomicOr(flags, kDup);
}

// By eid: the edge's position in a T order (the inverse of leid).
__global__ void tpos_kernel(const int32_t* leid, int64_t m, int32_t* pos) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p < m && (uint32_t)leid[p] < (uint64_t)m) pos[leid[p]] = (int32_t)p;
}

// N order: the packed key from the carried neighbour and time (ntime: the
// carried times, which may be nkey itself), and each entry's position in
// this direction's T order.
template <typename TT>
__global__ void n_order_fix_kernel(const uint32_t* nbr, const TT* ntime, const int32_t* neid, const int32_t* tpos,
                                   int64_t m, int bt, u64* nkey, int32_t* nxref) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= m) return;
    nkey[q] = ((u64)nbr[q] << bt) | (u64)ntime[q];
    nxref[q] = (uint32_t)neid[q] < (uint64_t)m ? tpos[neid[q]] : -1;
}

// (neighbour, time) records of a T order with 32-bit times.
__global__ void pack_nt_kernel(const uint32_t* nbr, const uint32_t* t, int64_t m, uint2* nt) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p < m) nt[p] = make_uint2(nbr[p], t[p]);
}

// List offsets from the owner-sorted keys: off[v] is the first position whose
// owner is >= v.  Position p writes the offsets of the owners in
// (key[p-1], key[p]]; the last position also closes the owners after it.
__global__ void offsets_kernel(const uint32_t* key, int64_t m, int32_t n, int32_t* off) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= m) return;
    // (owners are below n; the clamps keep a broken order from writing
    // outside off)
    const int64_t cur = key[p] < (uint32_t)n ? (int64_t)key[p] : (int64_t)n - 1;
    const int64_t prev = p == 0 ? -1 : (key[p - 1] < (uint32_t)n ? (int64_t)key[p - 1] : (int64_t)n - 1);
    for (int64_t v = prev + 1; v <= cur; ++v) off[v] = (int32_t)p;
    if (p == m - 1)
        for (int64_t v = cur + 1; v <= n; ++v) off[v] = (int32_t)m;
}

int bits_for(u64 x) {
    int b = 0;
    while (x) { ++b; x >>= 1; }
    return b;
}

unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

int graph_build(tm_graph* g, const int32_t* src, const int32_t* dst, const int64_t* t, hipStream_t st) {
    const int64_t m = g->m;
    const int32_t n = g->n;
    DevGraph& D = g->d;
    D.m = m;
    D.n = n;
    if (m == 0) {
        // empty graph: empty lists, every offset 0
        g->shift = 0;
        g->T = 0;
        D.T = 0;
        D.bt = 1;
        for (int dir = 0; dir < 2; ++dir) {
            int32_t* off;
            TM_TRY(arena_alloc(g->arena, &off, (size_t)n + 1));
            TM_HIP(hipMemsetAsync(off, 0, ((size_t)n + 1) * sizeof(int32_t), st));
            D.off[dir] = off;
        }
        TM_HIP(sync_stream(st));
        return TM_OK;
    }

    StageTimer timer;
    timer.start(TM_STAGE_GRAPH, st);
    // --- validation: ids, self loops, time span -------------------------
    int* flags = nullptr;
    u64* tbounds = nullptr;
    TM_HIP(dev_alloc((void**)&flags, sizeof(int) * 2, st));
    TM_HIP(dev_alloc((void**)&tbounds, sizeof(u64) * 2, st));
    TM_HIP(hipMemsetAsync(flags, 0, sizeof(int) * 2, st));
    {
        const unsigned blocks = (unsigned)std::min<int64_t>(grid_for(m), 1024);
        u64* part = nullptr;
        TM_HIP(dev_alloc((void**)&part, (size_t)blocks * 3 * sizeof(u64), st));
        hipLaunchKernelGGL(validate_kernel, dim3(blocks), dim3(kBlock), 0, st, src, dst, t, m, n, part);
        TM_HIP(hipGetLastError());
        hipLaunchKernelGGL(validate_reduce_kernel, dim3(1), dim3(kBlock), 0, st, (const u64*)part, (int)blocks,
                           flags, tbounds, tbounds + 1);
        TM_HIP(hipGetLastError());
        TM_HIP(dev_free(part, st));
    }
    // error exits return the flag words to the cache
    auto bail = [&](int r) {
        (void)dev_free(flags, st);
        (void)dev_free(tbounds, st);
        return r;
    };
    int hflags[2];
    u64 hb[2];
    TM_HIP(read_back({{hflags, flags, sizeof hflags}, {hb, tbounds, sizeof hb}}, st));
    if (hflags[0] & kBadRange) return bail(tm_fail(TM_EINVAL, "graph: vertex id outside [0, %d)", n));
    if (hflags[0] & kSelfLoop) return bail(tm_fail(TM_ESELFLOOP, "graph: self loop"));
    const int64_t tmin = (int64_t)(hb[0] ^ 0x8000000000000000ull);
    const int64_t tmax = (int64_t)(hb[1] ^ 0x8000000000000000ull);
    if ((__int128)tmax - (__int128)tmin >= ((__int128)1 << 62))
        return bail(tm_fail(TM_ERANGE, "graph: time span %lld..%lld too large", (long long)tmin, (long long)tmax));
    g->shift = tmin;
    g->T = tmax - tmin;
    D.T = g->T;
    const int bn = bits_for((u64)(n > 0 ? n - 1 : 0));
    D.bt = bits_for((u64)g->T);
    if (D.bt == 0) D.bt = 1;
    if (bn + D.bt > 64)
        return bail(tm_fail(TM_ERANGE, "graph: %d vertex-id bits + %d time bits exceed 64", bn, D.bt));

    // --- canonical order (t, u, v) ----------------------------------------
    // Four 64-bit work arrays serve every sort below: the canonical sorts use
    // them whole, the list sorts as halves.
    u64* work[4] = {nullptr, nullptr, nullptr, nullptr};
    uint32_t* nbr_tmp = nullptr;  // N order: the carried neighbours, when work[3] holds the owners
    // Lists keep their times in 32 bits when every shifted time is below
    // 2^32 - 1; t32e: those times by eid, the list sorts' input.
    const bool narrow = g->T < (int64_t)0xFFFFFFFFll;
    uint32_t* t32e = nullptr;
    uint32_t* nbr32[2] = {nullptr, nullptr};  // 32-bit times: the T orders' neighbours until packed
    auto release = [&]() {
        for (uint32_t*& b : nbr32) {
            if (b) (void)dev_free(b, st);
            b = nullptr;
        }
        for (u64*& w : work) {
            if (w) (void)dev_free(w, st);
            w = nullptr;
        }
        if (nbr_tmp) (void)dev_free(nbr_tmp, st);
        nbr_tmp = nullptr;
        if (t32e) (void)dev_free(t32e, st);
        t32e = nullptr;
    };
    int rc = TM_OK;
    for (u64*& w : work)
        if (rc == TM_OK && dev_alloc((void**)&w, (size_t)m * sizeof(u64), st) != hipSuccess)
            rc = tm_fail(TM_ENOMEM, "graph: work arrays");
    if (rc == TM_OK && narrow && dev_alloc((void**)&t32e, (size_t)m * sizeof(uint32_t), st) != hipSuccess)
        rc = tm_fail(TM_ENOMEM, "graph: work arrays");
    if (rc != TM_OK) {
        release();
        return bail(rc);
    }
    int32_t *esrc = nullptr, *edst = nullptr;
    int64_t* et = nullptr;
    rc = arena_alloc(g->arena, &esrc, m);
    if (rc == TM_OK) rc = arena_alloc(g->arena, &edst, m);
    if (rc == TM_OK) rc = arena_alloc(g->arena, &et, m);
    const bool one_key = 2 * bn + D.bt <= 64;
    if (rc == TM_OK) {
        hipLaunchKernelGGL(canon_keys_kernel, dim3(grid_for(m)), dim3(kBlock), 0, st, src, dst, t, m, tmin, bn,
                           one_key ? 1 : 0, work[0], work[1]);
        if (hipGetLastError() != hipSuccess) rc = tm_fail(TM_EDEVICE, "graph: key launch");
    }
    // A sort between two buffer sets: the result lands in `spare` after an
    // odd number of passes, else back in `in`.
    auto sort_two = [&](const auto& in, const auto& spare, int nbits, auto* res) -> int {
        const bool odd = (std::max(1, radix_passes(nbits)) & 1) != 0;
        *res = odd ? spare : in;
        return sort_into(in, odd ? spare : in, odd ? in : spare, m, 0, nbits, 0, flags + 1, st);
    };
    if (rc == TM_OK && one_key) {
        using S = SortSet<u64>;
        S in, spare, res;
        in.k = work[0];
        spare.k = work[2];
        rc = sort_two(in, spare, 2 * bn + D.bt, &res);
        if (rc == TM_OK)
            hipLaunchKernelGGL(decode_packed_kernel, dim3(grid_for(m)), dim3(kBlock), 0, st, (const u64*)res.k, m,
                               bn, esrc, edst, et, t32e, flags);
    } else if (rc == TM_OK) {
        // by (u, v) with the time carried, then by time with (u, v) carried
        using S = SortSet<u64, u64>;
        S x, y, r1, r2;
        x.k = work[0];
        x.v0 = work[1];
        y.k = work[2];
        y.v0 = work[3];
        rc = sort_two(x, y, 2 * bn, &r1);
        if (rc == TM_OK) {
            const S& o1 = r1.k == x.k ? y : x;
            S in2, spare2;
            in2.k = r1.v0;
            in2.v0 = r1.k;
            spare2.k = o1.k;
            spare2.v0 = o1.v0;
            rc = sort_two(in2, spare2, D.bt, &r2);
        }
        if (rc == TM_OK)
            hipLaunchKernelGGL(decode_split_kernel, dim3(grid_for(m)), dim3(kBlock), 0, st, (const u64*)r2.k,
                               (const u64*)r2.v0, m, bn, esrc, edst, et, t32e, flags);
    }
    if (rc == TM_OK && hipGetLastError() != hipSuccess) rc = tm_fail(TM_EDEVICE, "graph: decode launch");
    if (rc != TM_OK) {
        release();
        return bail(rc);
    }
    D.src = esrc;
    D.dst = edst;
    D.t = et;

    // --- per-vertex lists ---------------------------------------------------
    // dir 0: out-lists (owner = source, neighbour = destination)
    // dir 1: in-lists  (owner = destination, neighbour = source)
    // T order: the eids stably sorted by owner, carrying time, eid and
    // neighbour, so that every list array comes out of the sort in place.
    // TT: the lists' time type (uint32_t or int64_t).
    auto build_lists = [&](auto time_tag) -> int {
        using TT = decltype(time_tag);
        using V = typename std::conditional<sizeof(TT) == 4, uint32_t, u64>::type;
        using L = SortSet<uint32_t, V, uint32_t, uint32_t>;
        L tmp;  // the other buffer of the list sorts
        tmp.k = reinterpret_cast<uint32_t*>(work[0]);
        tmp.v1 = reinterpret_cast<uint32_t*>(work[0]) + m;
        tmp.v0 = reinterpret_cast<V*>(work[1]);
        tmp.v2 = reinterpret_cast<uint32_t*>(work[2]);
        uint32_t* nkeys_out = reinterpret_cast<uint32_t*>(work[2]) + m;  // N order: its sorted keys (unused)
        // N order: the carried times (32-bit: the upper half of work[1]; 64-bit:
        // the key array itself, packed in place afterwards)
        uint32_t* ntime32 = reinterpret_cast<uint32_t*>(work[1]) + m;
        const bool keep_own = m <= ((int64_t)1 << 28);
        uint32_t* own[2] = {nullptr, nullptr};
        if (!keep_own && dev_alloc((void**)&nbr_tmp, (size_t)m * sizeof(uint32_t), st) != hipSuccess)
            return tm_fail(TM_ENOMEM, "graph: work arrays");
        uint32_t* nbr_carried = keep_own ? reinterpret_cast<uint32_t*>(work[3]) : nbr_tmp;
        int32_t* tpos[2] = {nullptr, nullptr};
        TT* ltab[2] = {nullptr, nullptr};
        uint32_t* lnbr_of[2] = {nullptr, nullptr};  // each T order's neighbours (the N-order sorts' keys)
        for (int dir = 0; dir < 2; ++dir) {
            TT* lt = nullptr;
            int32_t *leid = nullptr, *lnbr = nullptr, *lown = nullptr, *off = nullptr;
            TM_TRY(arena_alloc(g->arena, &lt, m));
            TM_TRY(arena_alloc(g->arena, &leid, m));
            if constexpr (sizeof(TT) == 4) {
                // the neighbours end up in the (neighbour, time) records
                if (dev_alloc((void**)&nbr32[dir], (size_t)m * sizeof(uint32_t), st) != hipSuccess)
                    return tm_fail(TM_ENOMEM, "graph: work arrays");
                lnbr = reinterpret_cast<int32_t*>(nbr32[dir]);
            } else {
                TM_TRY(arena_alloc(g->arena, &lnbr, m));
            }
            if (keep_own) TM_TRY(arena_alloc(g->arena, &lown, m));
            TM_TRY(arena_alloc(g->arena, &off, (size_t)n + 1));
            TM_TRY(arena_alloc(g->arena, &tpos[dir], (size_t)m));
            own[dir] = keep_own ? reinterpret_cast<uint32_t*>(lown) : reinterpret_cast<uint32_t*>(work[3]) + dir * m;
            L in, out;
            in.k = reinterpret_cast<uint32_t*>(dir == 0 ? esrc : edst);
            in.v0 = sizeof(TT) == 4 ? reinterpret_cast<V*>(t32e) : reinterpret_cast<V*>(et);
            in.v2 = reinterpret_cast<uint32_t*>(dir == 0 ? edst : esrc);
            out.k = own[dir];
            out.v0 = reinterpret_cast<V*>(lt);
            out.v1 = reinterpret_cast<uint32_t*>(leid);
            out.v2 = reinterpret_cast<uint32_t*>(lnbr);
            TM_TRY(sort_into(in, out, tmp, m, 0, bn, 2 /* eids: 0, 1, ... */, flags + 1, st));
            hipLaunchKernelGGL(offsets_kernel, dim3(grid_for(m)), dim3(kBlock), 0, st, (const uint32_t*)own[dir],
                               m, n, off);
            hipLaunchKernelGGL(tpos_kernel, dim3(grid_for(m)), dim3(kBlock), 0, st, (const int32_t*)leid, m,
                               tpos[dir]);
            if (hipGetLastError() != hipSuccess) return tm_fail(TM_EDEVICE, "graph: list launch");
            D.off[dir] = off;
            D.tpos[dir] = tpos[dir];
            ltab[dir] = lt;
            if constexpr (sizeof(TT) == 4) {
                uint2* nt = nullptr;
                TM_TRY(arena_alloc(g->arena, &nt, m));
                hipLaunchKernelGGL(pack_nt_kernel, dim3(grid_for(m)), dim3(kBlock), 0, st,
                                   (const uint32_t*)lnbr, (const uint32_t*)lt, m, nt);
                if (hipGetLastError() != hipSuccess) return tm_fail(TM_EDEVICE, "graph: list launch");
                D.lt32[dir] = reinterpret_cast<const uint32_t*>(lt);
                D.lt[dir] = nullptr;
                D.lnt[dir] = nt;
                D.lnbr[dir] = nullptr;
            } else {
                D.lt[dir] = reinterpret_cast<const int64_t*>(lt);
                D.lt32[dir] = nullptr;
                D.lnt[dir] = nullptr;
                D.lnbr[dir] = lnbr;
            }
            lnbr_of[dir] = reinterpret_cast<uint32_t*>(lnbr);
            D.leid[dir] = leid;
            D.lown[dir] = lown;
        }
        // N order of dir d: the T order of the other direction (sorted by this
        // direction's neighbour, then time) stably re-sorted by this
        // direction's owner, carrying time, eid and neighbour.
        for (int dir = 0; dir < 2; ++dir) {
            const int other = 1 - dir;
            u64* nkey = nullptr;
            int32_t *nxref = nullptr, *neid = nullptr;
            TM_TRY(arena_alloc(g->arena, &nkey, m));
            TM_TRY(arena_alloc(g->arena, &nxref, m));
            TM_TRY(arena_alloc(g->arena, &neid, m));
            L in, out;
            in.k = lnbr_of[other];
            in.v0 = reinterpret_cast<V*>(ltab[other]);
            in.v1 = reinterpret_cast<uint32_t*>(const_cast<int32_t*>(D.leid[other]));
            in.v2 = own[other];
            out.k = nkeys_out;
            out.v0 = sizeof(TT) == 4 ? reinterpret_cast<V*>(ntime32) : reinterpret_cast<V*>(nkey);
            out.v1 = reinterpret_cast<uint32_t*>(neid);
            out.v2 = nbr_carried;
            TM_TRY(sort_into(in, out, tmp, m, 0, bn, 0, flags + 1, st));
            hipLaunchKernelGGL((n_order_fix_kernel<V>), dim3(grid_for(m)), dim3(kBlock), 0, st,
                               (const uint32_t*)nbr_carried, (const V*)out.v0, (const int32_t*)neid,
                               (const int32_t*)tpos[dir], m, D.bt, nkey, nxref);
            if (hipGetLastError() != hipSuccess) return tm_fail(TM_EDEVICE, "graph: list launch");
            D.nkey[dir] = nkey;
            D.nxref[dir] = nxref;
            D.neid[dir] = neid;
        }
        return TM_OK;
    };
    rc = narrow ? build_lists(uint32_t{}) : build_lists(int64_t{});
    release();
    if (rc != TM_OK) return bail(rc);
    timer.stop();
    TM_HIP(read_back({{hflags, flags, sizeof hflags}}, st));
    TM_HIP(dev_free(flags, st));
    TM_HIP(dev_free(tbounds, st));
    timer.finish();
    if (hflags[0] & kDup) return tm_fail(TM_EDUP, "graph: duplicate (u, v, t) tuple");
    if (hflags[1]) return tm_fail(TM_EDEVICE, "graph: internal sort error (look-back stalled)");
    return TM_OK;
}
