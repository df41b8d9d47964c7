// Graph build: validation, the canonical edge order and the per-vertex lists.
//
// The paper stores the graph as per-vertex in/out edge lists sorted by time,
// searched by binary search (Sec. 4, storage paragraph), with timestamps
// shifted to start at 0.  Here every list is built by stable LSD radix sorts
// so that the order inside each list is the canonical eid order.
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

// Sort keys for the canonical order (t, u, v).
__global__ void key_tuv_kernel(const int32_t* src, const int32_t* dst, const int64_t* t, int64_t m,
                               int64_t tmin, int bn, int with_time, u64* keys, uint32_t* vals) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= m) return;
    u64 k = ((u64)(uint32_t)src[i] << bn) | (u64)(uint32_t)dst[i];
    if (with_time) k |= (u64)(t[i] - tmin) << (2 * bn);
    keys[i] = k;
    vals[i] = (uint32_t)i;
}

__global__ void key_time_kernel(const int64_t* t, const uint32_t* perm, int64_t m, int64_t tmin,
                                u64* keys) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < m) keys[i] = (u64)(t[perm[i]] - tmin);
}

// Edge arrays in eid order, and the duplicate check on neighbours in that order.
__global__ void gather_edges_kernel(const int32_t* src, const int32_t* dst, const int64_t* t,
                                    const uint32_t* perm, int64_t m, int64_t tmin, int32_t* osrc,
                                    int32_t* odst, int64_t* ot, int* flags) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= m) return;
    const uint32_t i = perm[e];
    osrc[e] = src[i];
    odst[e] = dst[i];
    ot[e] = t[i] - tmin;
    if (e > 0) {
        const uint32_t j = perm[e - 1];
        if (src[i] == src[j] && dst[i] == dst[j] && t[i] == t[j]) atomicOr(flags, kDup);
    }
}

// Edge arrays straight from sorted packed keys t << 2bn | u << bn | v, and the
// duplicate check on neighbours.
__global__ void decode_edges_kernel(const u64* key, int64_t m, int bn, int32_t* osrc, int32_t* odst,
                                    int64_t* ot, int* flags) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= m) return;
    const u64 k = key[e];
    const u64 mask = (1ull << bn) - 1;
    osrc[e] = (int32_t)((k >> bn) & mask);
    odst[e] = (int32_t)(k & mask);
    ot[e] = (int64_t)(k >> (2 * bn));
    if (e > 0 && key[e - 1] == k) atomicOr(flags, kDup);
}

__global__ void iota_key_kernel(const int32_t* key_by_eid, int64_t m, uint32_t* keys, uint32_t* vals) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= m) return;
    keys[e] = (uint32_t)key_by_eid[e];
    vals[e] = (uint32_t)e;
}

__global__ void copy_pair_kernel(const int32_t* k, const int32_t* v, int64_t m, uint32_t* keys,
                                 uint32_t* vals) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= m) return;
    keys[p] = (uint32_t)k[p];
    vals[p] = (uint32_t)v[p];
}

// T-order list entries from the sorted eids.
__global__ void fill_t_order_kernel(const uint32_t* eids, const uint32_t* owner, const int64_t* t,
                                    const int32_t* nbr_by_eid, int64_t m, int64_t* lt, int32_t* leid, int32_t* lnbr,
                                    int32_t* lown, int32_t* pos) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= m) return;
    const uint32_t e = eids[p];
    lt[p] = t[e];
    leid[p] = (int32_t)e;
    lnbr[p] = nbr_by_eid[e];
    if (lown) lown[p] = (int32_t)owner[p];
    pos[e] = (int32_t)p;
}

// N-order list entries: packed (neighbour, time) key and the T-order position.
__global__ void fill_n_order_kernel(const uint32_t* eids, const int64_t* t, const int32_t* nbr_by_eid,
                                    const int32_t* tpos, int64_t m, int bt, u64* nkey, int32_t* nxref,
                                    int32_t* neid) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= m) return;
    const uint32_t e = eids[p];
    nkey[p] = ((u64)(uint32_t)nbr_by_eid[e] << bt) | (u64)t[e];
    nxref[p] = tpos[e];
    neid[p] = (int32_t)e;
}

// The same two fills reading one packed key t << 2bn | u << bn | v per eid
// (the canonical sort's output) instead of the separate edge arrays.
__device__ __forceinline__ void unpack_tuv(u64 k, int bn, int64_t& t, int32_t& u, int32_t& v) {
    const u64 mask = (1ull << bn) - 1;
    t = (int64_t)(k >> (2 * bn));
    u = (int32_t)((k >> bn) & mask);
    v = (int32_t)(k & mask);
}

__global__ void fill_t_order_packed_kernel(const uint32_t* eids, const u64* pk, int bn, int dir, int64_t m,
                                           int64_t* lt, int32_t* leid, int32_t* lnbr, int32_t* lown, int32_t* pos) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= m) return;
    const uint32_t e = eids[p];
    int64_t t;
    int32_t u, v;
    unpack_tuv(pk[e], bn, t, u, v);
    lt[p] = t;
    leid[p] = (int32_t)e;
    lnbr[p] = dir == 0 ? v : u;
    if (lown) lown[p] = dir == 0 ? u : v;
    pos[e] = (int32_t)p;
}

__global__ void fill_n_order_packed_kernel(const uint32_t* eids, const u64* pk, int bn, int dir,
                                           const int32_t* tpos, int64_t m, int bt, u64* nkey, int32_t* nxref,
                                           int32_t* neid) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= m) return;
    const uint32_t e = eids[p];
    int64_t t;
    int32_t u, v;
    unpack_tuv(pk[e], bn, t, u, v);
    nkey[p] = ((u64)(uint32_t)(dir == 0 ? v : u) << bt) | (u64)t;
    nxref[p] = tpos[e];
    neid[p] = (int32_t)e;
}

// List offsets from the owner-sorted keys: off[v] is the first position whose
// owner is >= v.  Position p writes the offsets of the owners in
// (key[p-1], key[p]]; the last position also closes the owners after it.
__global__ void offsets_kernel(const uint32_t* key, int64_t m, int32_t n, int32_t* off) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= m) return;
    const int64_t cur = key[p];
    const int64_t prev = p == 0 ? -1 : (int64_t)key[p - 1];
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
    int hflags[2];
    u64 hb[2];
    TM_HIP(read_back({{hflags, flags, sizeof hflags}, {hb, tbounds, sizeof hb}}, st));
    if (hflags[0] & kBadRange) return tm_fail(TM_EINVAL, "graph: vertex id outside [0, %d)", n);
    if (hflags[0] & kSelfLoop) return tm_fail(TM_ESELFLOOP, "graph: self loop");
    const int64_t tmin = (int64_t)(hb[0] ^ 0x8000000000000000ull);
    const int64_t tmax = (int64_t)(hb[1] ^ 0x8000000000000000ull);
    if ((__int128)tmax - (__int128)tmin >= ((__int128)1 << 62))
        return tm_fail(TM_ERANGE, "graph: time span %lld..%lld too large", (long long)tmin,
                       (long long)tmax);
    g->shift = tmin;
    g->T = tmax - tmin;
    D.T = g->T;
    const int bn = bits_for((u64)(n > 0 ? n - 1 : 0));
    D.bt = bits_for((u64)g->T);
    if (D.bt == 0) D.bt = 1;
    if (bn + D.bt > 64)
        return tm_fail(TM_ERANGE, "graph: %d vertex-id bits + %d time bits exceed 64", bn, D.bt);

    // --- canonical order (t, u, v) ----------------------------------------
    u64 *ka = nullptr, *kb = nullptr;
    uint32_t *va = nullptr, *vb = nullptr;
    TM_HIP(dev_alloc((void**)&ka, m * sizeof(u64), st));
    TM_HIP(dev_alloc((void**)&kb, m * sizeof(u64), st));
    TM_HIP(dev_alloc((void**)&va, m * sizeof(uint32_t), st));
    TM_HIP(dev_alloc((void**)&vb, m * sizeof(uint32_t), st));
    u64* kres;
    uint32_t* perm;
    const bool one_key = 2 * bn + D.bt <= 64;
    hipLaunchKernelGGL(key_tuv_kernel, dim3(grid_for(m)), dim3(kBlock), 0, st, src, dst, t, m, tmin,
                       bn, one_key ? 1 : 0, ka, va);
    TM_HIP(hipGetLastError());
    if (one_key) {
        TM_TRY(radix_sort_pairs<u64>(ka, va, kb, vb, m, 0, 2 * bn + D.bt, &kres, &perm, flags + 1, st));
    } else {
        TM_TRY(radix_sort_pairs<u64>(ka, va, kb, vb, m, 0, 2 * bn, &kres, &perm, flags + 1, st));
        u64* kother = kres == ka ? kb : ka;
        uint32_t* vother = perm == va ? vb : va;
        hipLaunchKernelGGL(key_time_kernel, dim3(grid_for(m)), dim3(kBlock), 0, st, t, perm, m,
                           tmin, kother);
        TM_HIP(hipGetLastError());
        TM_TRY(radix_sort_pairs<u64>(kother, perm, kres, vother, m, 0, D.bt, &kres, &perm, flags + 1,
                                     st));
    }
    int32_t *esrc, *edst;
    int64_t* et;
    TM_TRY(arena_alloc(g->arena, &esrc, m));
    TM_TRY(arena_alloc(g->arena, &edst, m));
    TM_TRY(arena_alloc(g->arena, &et, m));
    if (one_key && bn > 0)
        hipLaunchKernelGGL(decode_edges_kernel, dim3(grid_for(m)), dim3(kBlock), 0, st,
                           (const u64*)kres, m, bn, esrc, edst, et, flags);
    else
        hipLaunchKernelGGL(gather_edges_kernel, dim3(grid_for(m)), dim3(kBlock), 0, st, src, dst, t,
                           (const uint32_t*)perm, m, tmin, esrc, edst, et, flags);
    TM_HIP(hipGetLastError());
    D.src = esrc;
    D.dst = edst;
    D.t = et;

    // --- per-vertex lists ---------------------------------------------------
    // dir 0: out-lists (key = source, neighbour = destination)
    // dir 1: in-lists  (key = destination, neighbour = source)
    // with one packed key per edge, the sorted keys stay for the fills and
    // the other key buffer holds both 32-bit key buffers of the list sorts
    const bool packed = one_key && bn > 0;
    u64* kspare = kres == ka ? kb : ka;
    uint32_t* k32a = reinterpret_cast<uint32_t*>(packed ? kspare : ka);
    uint32_t* k32b = packed ? k32a + m : reinterpret_cast<uint32_t*>(kb);
    int32_t* tpos[2];
    for (int dir = 0; dir < 2; ++dir) {
        const int32_t* key_by_eid = dir == 0 ? esrc : edst;
        const int32_t* nbr_by_eid = dir == 0 ? edst : esrc;
        int64_t* lt;
        int32_t *leid, *lnbr, *lown, *off;
        TM_TRY(arena_alloc(g->arena, &lt, m));
        TM_TRY(arena_alloc(g->arena, &leid, m));
        TM_TRY(arena_alloc(g->arena, &lnbr, m));
        lown = nullptr;
        if (m <= ((int64_t)1 << 28)) TM_TRY(arena_alloc(g->arena, &lown, m));
        TM_TRY(arena_alloc(g->arena, &off, (size_t)n + 1));
        TM_TRY(arena_alloc(g->arena, &tpos[dir], (size_t)m));
        // T order: stable sort of the eids by the list owner
        hipLaunchKernelGGL(iota_key_kernel, dim3(grid_for(m)), dim3(kBlock), 0, st, key_by_eid, m,
                           k32a, va);
        TM_HIP(hipGetLastError());
        uint32_t *kr, *vr;
        TM_TRY(radix_sort_pairs<uint32_t>(k32a, va, k32b, vb, m, 0, bn, &kr, &vr, flags + 1, st));
        if (packed)
            hipLaunchKernelGGL(fill_t_order_packed_kernel, dim3(grid_for(m)), dim3(kBlock), 0, st,
                               (const uint32_t*)vr, (const u64*)kres, bn, dir, m, lt, leid, lnbr, lown, tpos[dir]);
        else
            hipLaunchKernelGGL(fill_t_order_kernel, dim3(grid_for(m)), dim3(kBlock), 0, st,
                               (const uint32_t*)vr, (const uint32_t*)kr, (const int64_t*)et, nbr_by_eid, m, lt,
                               leid, lnbr, lown, tpos[dir]);
        TM_HIP(hipGetLastError());
        hipLaunchKernelGGL(offsets_kernel, dim3(grid_for(m)), dim3(kBlock), 0, st,
                           (const uint32_t*)kr, m, n, off);
        TM_HIP(hipGetLastError());
        D.off[dir] = off;
        D.tpos[dir] = tpos[dir];
        D.lt[dir] = lt;
        D.leid[dir] = leid;
        D.lown[dir] = lown;
        D.lnbr[dir] = lnbr;
    }
    // N order of dir d: the T order of the other direction (sorted by the
    // neighbour, then time) stably re-sorted by this direction's owner.
    for (int dir = 0; dir < 2; ++dir) {
        const int other = 1 - dir;
        const int32_t* nbr_by_eid = dir == 0 ? edst : esrc;
        u64* nkey;
        int32_t *nxref, *neid;
        TM_TRY(arena_alloc(g->arena, &nkey, m));
        TM_TRY(arena_alloc(g->arena, &nxref, m));
        TM_TRY(arena_alloc(g->arena, &neid, m));
        // keys: the owner of each entry of the other direction's T order,
        // which is that entry's neighbour there
        hipLaunchKernelGGL(copy_pair_kernel, dim3(grid_for(m)), dim3(kBlock), 0, st,
                           D.lnbr[other], D.leid[other], m, k32a, va);
        TM_HIP(hipGetLastError());
        uint32_t *kr, *vr;
        TM_TRY(radix_sort_pairs<uint32_t>(k32a, va, k32b, vb, m, 0, bn, &kr, &vr, flags + 1, st));
        if (packed)
            hipLaunchKernelGGL(fill_n_order_packed_kernel, dim3(grid_for(m)), dim3(kBlock), 0, st,
                               (const uint32_t*)vr, (const u64*)kres, bn, dir, (const int32_t*)tpos[dir], m, D.bt,
                               nkey, nxref, neid);
        else
            hipLaunchKernelGGL(fill_n_order_kernel, dim3(grid_for(m)), dim3(kBlock), 0, st,
                               (const uint32_t*)vr, (const int64_t*)et, nbr_by_eid,
                               (const int32_t*)tpos[dir], m, D.bt, nkey, nxref, neid);
        TM_HIP(hipGetLastError());
        D.nkey[dir] = nkey;
        D.nxref[dir] = nxref;
        D.neid[dir] = neid;
    }
    TM_HIP(dev_free(ka, st));
    TM_HIP(dev_free(kb, st));
    TM_HIP(dev_free(va, st));
    TM_HIP(dev_free(vb, st));
    timer.stop();
    TM_HIP(read_back({{hflags, flags, sizeof hflags}}, st));
    TM_HIP(dev_free(flags, st));
    TM_HIP(dev_free(tbounds, st));
    timer.finish();
    if (hflags[0] & kDup) return tm_fail(TM_EDUP, "graph: duplicate (u, v, t) tuple");
    if (hflags[1]) return tm_fail(TM_EDEVICE, "graph: internal scan overflow");
    return TM_OK;
}
