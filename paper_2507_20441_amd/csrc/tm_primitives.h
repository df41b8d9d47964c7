// Device-wide primitives of the TIMEST GPU library: exclusive prefix sums and
// a stable LSD radix sort of (key, value) pairs.  Templates, instantiated by
// the translation units that use them.
#pragma once

#include <algorithm>
#include <type_traits>

#include "tm_internal.h"

constexpr int kScanItems = 8;                      // values per lane in a scan tile
constexpr int kScanTile = kBlock * kScanItems;     // 2048
constexpr int kSortBits = 8;                       // sort digits: up to 8 bits, one per lane
constexpr int kSortDigits = 1 << kSortBits;        // 256
constexpr int kSortItems = 16;                     // keys per lane in a sort tile
constexpr int kSortTile = kBlock * kSortItems;     // 4096
constexpr int kSortMaxPasses = 8;
static_assert(kSortDigits == kBlock, "one digit per lane of a block");

// Radix passes over nb key bits (digits of at most kSortBits, split as
// evenly as possible).
inline int radix_passes(int nb) { return nb <= 0 ? 0 : (nb + kSortBits - 1) / kSortBits; }

// Clearing device words with a kernel rather than a memset node, so that the
// same code can be captured into a HIP graph.
__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v);
// p[i] = i for i < n.
int fill_iota_u32(uint32_t* p, int64_t n, hipStream_t st);

// ---------------------------------------------------------------------------
// Wave and block scans of 128-bit values (two 64-bit shuffles per step).
// ---------------------------------------------------------------------------
__device__ __forceinline__ u128 shfl_up_u128(u128 v, int d) {
    u64 lo = __shfl_up((u64)v, d, 64);
    u64 hi = __shfl_up((u64)(v >> 64), d, 64);
    return ((u128)hi << 64) | lo;
}

// Inclusive scan across the 64 lanes of a wave; sets *carry on wrap-around.
__device__ __forceinline__ u128 wave_inclusive(u128 v, int lane, bool* carry) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        u128 o = shfl_up_u128(v, d);
        if (lane >= d) {
            u128 s = v + o;
            if (s < v) *carry = true;
            v = s;
        }
    }
    return v;
}

// Exclusive scan over the block's 256 lanes; returns the lane's exclusive
// prefix and writes the block total.  Uses a small LDS array.
__device__ __forceinline__ u128 block_exclusive(u128 v, u128* total, bool* carry) {
    __shared__ u128 wsum[kWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    u128 inc = wave_inclusive(v, lane, carry);
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    u128 before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        u128 x = wsum[w];
        if (w < wave) before += x;
        u128 s = all + x;
        if (s < all) *carry = true;
        all = s;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

// ---------------------------------------------------------------------------
// Exclusive scan: out[i] = sum of f(0..i-1) for i = 0..n (out[n] = total).
// Accumulation is exact in 128 bits; out is written in T.  Every output is
// exact when the total fits T; otherwise bit 1 of *ovf is set.  A 128-bit
// wrap sets bit 0.
// Reduce-then-scan: tile sums, a scan of the tile sums, then each tile.
// ---------------------------------------------------------------------------
template <typename F>
__global__ void __launch_bounds__(kBlock) scan_tiles_kernel(F f, int64_t n, u128* part, int* ovf) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    u128 s = 0;
    bool carry = false;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
        if (i < n) {
            u128 x = to_u128(f(i));
            u128 y = s + x;
            if (y < s) carry = true;
            s = y;
        }
    }
    u128 tot;
    block_exclusive(s, &tot, &carry);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
    if (carry) atomicOr(ovf, 1);
}

template <typename T, typename F>
__global__ void __launch_bounds__(kBlock)
scan_apply_kernel(F f, int64_t n, const u128* part_scan, T* out, int* ovf) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    // each lane owns kScanItems consecutive values of the tile
    const int64_t first = base + (int64_t)threadIdx.x * kScanItems;
    u128 v[kScanItems];
    u128 s = 0;
    bool carry = false;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = first + k;
        v[k] = i < n ? to_u128(f(i)) : (u128)0;
        u128 y = s + v[k];
        if (y < s) carry = true;
        s = y;
    }
    u128 tot;
    u128 run = part_scan[blockIdx.x] + block_exclusive(s, &tot, &carry);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = first + k;
        if (i < n) out[i] = (T)run;
        u128 y = run + v[k];
        if (y < run) carry = true;
        run = y;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        const u128 total = part_scan[gridDim.x];
        out[n] = (T)total;
        if ((u128)(T)total != total) atomicOr(ovf, 2);  // total does not fit T
    }
    if (carry) atomicOr(ovf, 1);
}

struct ArrayReader128 {
    const u128* a;
    __device__ u128 operator()(int64_t i) const { return a[i]; }
};

// Exclusive scan of the tile sums in place: part[0..nb] (part[nb] = total).
int scan_parts(u128* part, int64_t nb, int* ovf, hipStream_t st);

template <typename T, typename F>
int device_exclusive_scan(F f, int64_t n, T* out, int* ovf, hipStream_t st) {
    if (n == 0) {
        static_assert(sizeof(T) % 4 == 0, "scan outputs are whole words");
        return fill_u32(out, sizeof(T) / 4, 0u, st);
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    u128* part = nullptr;
    TM_HIP(dev_alloc((void**)&part, (nb + 1) * sizeof(u128), st));
    hipLaunchKernelGGL((scan_tiles_kernel<F>), dim3((unsigned)nb), dim3(kBlock), 0, st, f, n, part,
                       ovf);
    TM_HIP(hipGetLastError());
    int rc = scan_parts(part, nb, ovf, st);
    if (rc == TM_OK) {
        hipLaunchKernelGGL((scan_apply_kernel<T, F>), dim3((unsigned)nb), dim3(kBlock), 0, st, f,
                           n, (const u128*)part, out, ovf);
        TM_HIP(hipGetLastError());
    }
    TM_HIP(dev_free(part, st));
    return rc;
}

// ---------------------------------------------------------------------------
// Two exclusive scans in one pass: f(i) returns the i-th value of both
// sequences (a Pair2), so a record holding both is read once.  Same outputs
// and flags as two device_exclusive_scan calls.
// ---------------------------------------------------------------------------
template <typename V>
struct Pair2 {
    V a, b;
};

template <typename F>
__global__ void __launch_bounds__(kBlock) scan2_tiles_kernel(F f, int64_t n, u128* part0, u128* part1, int* ovf) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    u128 s0 = 0, s1 = 0;
    bool carry = false;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
        if (i < n) {
            const auto x = f(i);
            const u128 y0 = s0 + to_u128(x.a), y1 = s1 + to_u128(x.b);
            if (y0 < s0 || y1 < s1) carry = true;
            s0 = y0;
            s1 = y1;
        }
    }
    u128 tot0, tot1;
    block_exclusive(s0, &tot0, &carry);
    block_exclusive(s1, &tot1, &carry);
    if (threadIdx.x == 0) {
        part0[blockIdx.x] = tot0;
        part1[blockIdx.x] = tot1;
    }
    if (carry) atomicOr(ovf, 1);
}

template <typename T, typename F>
__global__ void __launch_bounds__(kBlock)
scan2_apply_kernel(F f, int64_t n, const u128* part0, const u128* part1, T* out0, T* out1, int* ovf) {
    using V = decltype(f(0).a);
    // Values come in and results go out in rounds of kBlock consecutive
    // entries (coalesced), through LDS; in between each lane scans a run of
    // kScanItems consecutive entries.  Entry j of the tile sits at LDS
    // position j + j / kScanItems, so that the lanes reading their runs do
    // not all fall on the same banks.
    constexpr int kPad = kScanTile + kScanTile / kScanItems;
    constexpr size_t kElt = sizeof(V) > sizeof(T) ? sizeof(V) : sizeof(T);
    __shared__ __align__(16) unsigned char sbuf[2 * kPad * kElt];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    V* lv0 = reinterpret_cast<V*>(sbuf);
    V* lv1 = lv0 + kPad;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int j = k * kBlock + (int)threadIdx.x;
        const int64_t i = base + j;
        V a = 0, b = 0;
        if (i < n) {
            const auto x = f(i);
            a = x.a;
            b = x.b;
        }
        lv0[j + j / kScanItems] = a;
        lv1[j + j / kScanItems] = b;
    }
    __syncthreads();
    u128 v0[kScanItems], v1[kScanItems];
    u128 s0 = 0, s1 = 0;
    bool carry = false;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int j = (int)threadIdx.x * kScanItems + k;
        v0[k] = to_u128(lv0[j + j / kScanItems]);
        v1[k] = to_u128(lv1[j + j / kScanItems]);
        const u128 y0 = s0 + v0[k], y1 = s1 + v1[k];
        if (y0 < s0 || y1 < s1) carry = true;
        s0 = y0;
        s1 = y1;
    }
    u128 tot0, tot1;
    u128 run0 = part0[blockIdx.x] + block_exclusive(s0, &tot0, &carry);
    u128 run1 = part1[blockIdx.x] + block_exclusive(s1, &tot1, &carry);
    __syncthreads();  // every lane has read its values: the buffer takes the results
    T* lo0 = reinterpret_cast<T*>(sbuf);
    T* lo1 = lo0 + kPad;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int j = (int)threadIdx.x * kScanItems + k;
        lo0[j + j / kScanItems] = (T)run0;
        lo1[j + j / kScanItems] = (T)run1;
        const u128 y0 = run0 + v0[k], y1 = run1 + v1[k];
        if (y0 < run0 || y1 < run1) carry = true;
        run0 = y0;
        run1 = y1;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int j = k * kBlock + (int)threadIdx.x;
        const int64_t i = base + j;
        if (i < n) {
            out0[i] = lo0[j + j / kScanItems];
            out1[i] = lo1[j + j / kScanItems];
        }
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        const u128 t0 = part0[gridDim.x], t1 = part1[gridDim.x];
        out0[n] = (T)t0;
        out1[n] = (T)t1;
        if ((u128)(T)t0 != t0 || (u128)(T)t1 != t1) atomicOr(ovf, 2);  // a total does not fit T
    }
    if (carry) atomicOr(ovf, 1);
}

template <typename T, typename F>
int device_exclusive_scan2(F f, int64_t n, T* out0, T* out1, int* ovf, hipStream_t st) {
    if (n == 0) {
        static_assert(sizeof(T) % 4 == 0, "scan outputs are whole words");
        TM_TRY(fill_u32(out0, sizeof(T) / 4, 0u, st));
        return fill_u32(out1, sizeof(T) / 4, 0u, st);
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    u128* part = nullptr;
    TM_HIP(dev_alloc((void**)&part, 2 * (nb + 1) * sizeof(u128), st));
    u128* part1 = part + nb + 1;
    hipLaunchKernelGGL((scan2_tiles_kernel<F>), dim3((unsigned)nb), dim3(kBlock), 0, st, f, n, part, part1, ovf);
    TM_HIP(hipGetLastError());
    int rc = scan_parts(part, nb, ovf, st);
    if (rc == TM_OK) rc = scan_parts(part1, nb, ovf, st);
    if (rc == TM_OK) {
        hipLaunchKernelGGL((scan2_apply_kernel<T, F>), dim3((unsigned)nb), dim3(kBlock), 0, st, f, n,
                           (const u128*)part, (const u128*)part1, out0, out1, ovf);
        TM_HIP(hipGetLastError());
    }
    TM_HIP(dev_free(part, st));
    return rc;
}

// Exclusive scan of v over the block's 256 threads (thread t holds entry t):
// shuffles inside each wave, then the wave totals through LDS.
__device__ __forceinline__ uint32_t block_excl_scan_256(uint32_t v, uint32_t* wsum) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(inc, d, 64);
        if (lane >= d) inc += o;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t before = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) before += w < wave ? wsum[w] : 0u;
    __syncthreads();
    return before + inc - v;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of keys that carry up to three value arrays
// (structure of arrays), one kernel per digit of up to 8 bits:
//  * sort_hist_kernel counts the digits of every pass in one read of the
//    keys, and sort_base_kernel turns those counts into each digit's first
//    position;
//  * sort_pass_kernel, once per pass: a block takes the next tile by ticket
//    (so a tile only ever waits on tiles that are already running), ranks
//    its keys by digit with wave ballots, publishes its digit counts, and
//    finds where its run of each digit starts by adding up the counts that
//    the tiles before it published, back to a tile that has published its
//    inclusive total (decoupled look-back).  Keys and values then go out
//    through LDS, each digit's run of the tile to consecutive addresses.
// A status word holds a value (bits 0-31), a flag (bits 32-33: 1 the tile's
// own count, 2 the total through the tile) and the pass's tag (bits 40-47).
// The words are cleared once per sort, so a word left by an earlier pass
// reads as not yet published.  Waits are bounded: a lane that has polled
// kSortMaxSpins times sets kSortStall in the caller's error word and goes on
// (the order is then wrong, and the caller reports the error).
// ---------------------------------------------------------------------------
struct SortNone {};  // an absent value array
constexpr int kSortStall = 4;
constexpr uint32_t kSortMaxSpins = 1u << 20;
constexpr int kSortLook = 8;  // status words a look-back step reads
constexpr size_t kSortHeadBytes =
    ((size_t)kSortMaxPasses * kSortDigits * sizeof(uint32_t) + kSortMaxPasses * sizeof(uint32_t) + 255) &
    ~(size_t)255;

// Scratch of a sort of n keys: per-pass digit counts and tickets, then one
// status word per tile and digit.
constexpr size_t sort_scratch_bytes(int64_t n) {
    return kSortHeadBytes + (size_t)(n > 0 ? (n + kSortTile - 1) / kSortTile : 0) * kSortDigits * sizeof(u64);
}

struct SortPlan {
    int npass;
    int shift[kSortMaxPasses];
    int bits[kSortMaxPasses];
};

// Digits over bits [lo_bit, nbits), as even as possible; no pass when the
// range is empty.
inline SortPlan sort_plan(int lo_bit, int nbits) {
    SortPlan P{};
    P.npass = radix_passes(nbits - lo_bit);
    int shift = lo_bit;
    for (int p = 0; p < P.npass; ++p) {
        const int b = (nbits - shift + (P.npass - p) - 1) / (P.npass - p);
        P.shift[p] = shift;
        P.bits[p] = b;
        shift += b;
    }
    return P;
}

template <typename V>
struct SortSize {
    static constexpr size_t value = sizeof(V);
};
template <>
struct SortSize<SortNone> {
    static constexpr size_t value = 0;
};

struct SortIO {
    const void* in[4];  // keys, then the value arrays
    void* out[4];
};

template <typename K>
__global__ void __launch_bounds__(kBlock)
sort_hist_kernel(const K* __restrict__ keys, int64_t n, SortPlan P, uint32_t* __restrict__ ghist) {
    __shared__ uint32_t h[kSortMaxPasses][kSortDigits];
#pragma unroll
    for (int p = 0; p < kSortMaxPasses; ++p) h[p][threadIdx.x] = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const K k = keys[i];
        for (int p = 0; p < P.npass; ++p)
            atomicAdd(&h[p][(uint32_t)(k >> P.shift[p]) & ((1u << P.bits[p]) - 1u)], 1u);
    }
    __syncthreads();
    for (int p = 0; p < P.npass; ++p) {
        const uint32_t c = h[p][threadIdx.x];
        if (c) atomicAdd(&ghist[p * kSortDigits + threadIdx.x], c);
    }
}

// Each pass's digit counts, in place, into exclusive digit starts.
__global__ void __launch_bounds__(kBlock) sort_base_kernel(uint32_t* ghist, int npass);

// One value array of a tile through LDS to the positions of its keys.
template <typename V>
__device__ __forceinline__ void sort_move_values(const void* vin, void* vout, bool iota, int64_t wbase, int lane,
                                                 int64_t n, const uint32_t (&lp)[kSortItems], unsigned char* sbuf,
                                                 const uint8_t* sdig, const uint32_t* gofs, int tn) {
    if constexpr (!std::is_same<V, SortNone>::value) {
        V* sv = reinterpret_cast<V*>(sbuf);
        const V* in = static_cast<const V*>(vin);
        V* out = static_cast<V*>(vout);
        V x[kSortItems];
        const int64_t tbase = wbase - (int64_t)(threadIdx.x >> 6) * 64 * kSortItems;
        if (!iota && tbase + kSortTile <= n) {
            // a whole tile: one base address, the items at fixed offsets
            const V* vp = in + wbase + lane;
#pragma unroll
            for (int k = 0; k < kSortItems; ++k) x[k] = vp[k * 64];
        } else {
#pragma unroll
            for (int k = 0; k < kSortItems; ++k) {
                const int64_t i = wbase + (int64_t)k * 64 + lane;
                x[k] = i < n ? (iota ? (V)i : in[i]) : (V)0;
            }
        }
        __syncthreads();  // the buffer's previous contents have gone out
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) {
            const int64_t i = wbase + (int64_t)k * 64 + lane;
            if (i < n) sv[lp[k]] = x[k];
        }
        __syncthreads();
        for (int p = threadIdx.x; p < tn; p += kBlock) {
            const uint32_t g = gofs[sdig[p]] + (uint32_t)p;
            if ((int64_t)g < n) out[g] = sv[p];
        }
    }
}

template <typename K, typename V0, typename V1, typename V2>
__global__ void __launch_bounds__(kBlock)
sort_pass_kernel(SortIO io, int64_t n, int shift, int bits, uint32_t tag, int iota, const uint32_t* __restrict__ starts,
                 uint32_t* __restrict__ ticket, u64* __restrict__ status, int* __restrict__ err) {
    constexpr size_t kElt = std::max(std::max(sizeof(K), SortSize<V0>::value),
                                     std::max(SortSize<V1>::value, SortSize<V2>::value));
    __shared__ __align__(16) unsigned char sbuf[kElt * kSortTile];
    __shared__ uint8_t sdig[kSortTile];
    // per wave and digit: counts, then tile-local starts, at most kSortTile
    // (16 bits keep a 64-bit-key pass within four workgroups' LDS per CU)
    __shared__ uint16_t cnt[kWaves][kSortDigits];
    __shared__ uint32_t gofs[kSortDigits];  // per digit: its global position minus its tile-local one
    __shared__ uint32_t wsum[kWaves];
    __shared__ uint32_t s_tile;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
#pragma unroll
    for (int w = 0; w < kWaves; ++w) cnt[w][threadIdx.x] = 0;
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t tbase = (int64_t)tile * kSortTile;
    // wave w owns tile positions [w 64 kSortItems, (w + 1) 64 kSortItems), in
    // rounds of 64 consecutive keys: the wave ranks its keys in input order
    const int64_t wbase = tbase + (int64_t)wave * 64 * kSortItems;
    const uint32_t mask = (1u << bits) - 1u;
    const u64 lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const K* keys = static_cast<const K*>(io.in[0]);
    K key[kSortItems];
    uint32_t lp[kSortItems];  // (the digits are recomputed from the keys: fewer registers)
    if (tbase + kSortTile <= n) {
        // a whole tile: one base address, the items at fixed offsets
        const K* kp = keys + wbase + lane;
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) key[k] = kp[k * 64];
    } else {
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) {
            const int64_t i = wbase + (int64_t)k * 64 + lane;
            key[k] = i < n ? keys[i] : (K)0;
        }
    }
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t i = wbase + (int64_t)k * 64 + lane;
        const bool ok = i < n;
        const uint32_t d = ok ? ((uint32_t)(key[k] >> shift) & mask) : 0u;
        u64 peers = __ballot(ok);
        for (int b = 0; b < bits; ++b) {
            const u64 bal = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t before = cnt[wave][d];
        lp[k] = before + (uint32_t)__popcll(peers & lt_mask);
        // the lowest lane of each digit group advances the wave's counter
        if (ok && (peers & lt_mask) == 0) cnt[wave][d] = (uint16_t)(before + (uint32_t)__popcll(peers));
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // lane d: the tile's count of digit d, published at once (the first tile
    // publishes it as its inclusive total)
    const uint32_t d = threadIdx.x;
    uint32_t tcount = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) tcount += cnt[w][d];
    u64* my = status + (size_t)tile * kSortDigits + d;
    const u64 tagw = (u64)tag << 40;
    if (d <= mask)
        __hip_atomic_store(my, tagw | ((u64)(tile == 0 ? 2 : 1) << 32) | tcount, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    // tile-local starts: of each digit, and of each wave's keys inside it
    const uint32_t dstart = block_excl_scan_256(tcount, wsum);
    {
        uint32_t run = dstart;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t c = cnt[w][d];
            cnt[w][d] = (uint16_t)run;
            run += c;
        }
    }
    __syncthreads();
    K* skey = reinterpret_cast<K*>(sbuf);
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t i = wbase + (int64_t)k * 64 + lane;
        if (i < n) {
            const uint32_t dk = (uint32_t)(key[k] >> shift) & mask;  // the digit again
            const uint32_t p = cnt[wave][dk] + lp[k];
            lp[k] = p;
            skey[p] = key[k];
            sdig[p] = (uint8_t)dk;
        }
    }
    // look-back: the digit's count over all earlier tiles, kSortLook status
    // words per step (their loads in flight together), back to a tile that
    // has published its inclusive total
    if (d <= mask) {
        uint32_t excl = 0;
        if (tile > 0) {
            int64_t j = (int64_t)tile - 1;  // the nearest tile not yet added
            uint32_t spins = 0;
            while (true) {
                u64 sw[kSortLook];
#pragma unroll
                for (int i = 0; i < kSortLook; ++i) {
                    const int64_t x = j - i;
                    // before tile 0: an inclusive total of 0
                    sw[i] = x >= 0 ? __hip_atomic_load(status + (size_t)x * kSortDigits + d, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT)
                                   : tagw | ((u64)2 << 32);
                }
                int used = 0;
                bool done = false;
#pragma unroll
                for (int i = 0; i < kSortLook; ++i) {
                    if (done || used < i) continue;  // stopped before i
                    const uint32_t f = (uint32_t)(sw[i] >> 32) & 3u;
                    if ((uint32_t)(sw[i] >> 40) != tag || f == 0) continue;  // not published yet: poll again
                    excl += (uint32_t)sw[i];
                    used = i + 1;
                    done = f == 2;
                }
                if (done) break;
                j -= used;
                if (used == 0) {
                    if (++spins >= kSortMaxSpins) {
                        atomicOr(err, kSortStall);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            __hip_atomic_store(my, tagw | ((u64)2 << 32) | (u64)(excl + tcount), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        gofs[d] = starts[d] + excl - dstart;
    }
    __syncthreads();
    const int tn = (int)(n - tbase < kSortTile ? n - tbase : kSortTile);
    K* okeys = static_cast<K*>(io.out[0]);
    // (positions are below n whenever the digit counts hold; the test keeps
    // a broken invariant from writing outside the output)
    for (int p = threadIdx.x; p < tn; p += kBlock) {
        const uint32_t g = gofs[sdig[p]] + (uint32_t)p;
        if ((int64_t)g < n) okeys[g] = skey[p];
    }
    sort_move_values<V0>(io.in[1], io.out[1], iota & 1, wbase, lane, n, lp, sbuf, sdig, gofs, tn);
    sort_move_values<V1>(io.in[2], io.out[2], iota & 2, wbase, lane, n, lp, sbuf, sdig, gofs, tn);
    sort_move_values<V2>(io.in[3], io.out[3], iota & 4, wbase, lane, n, lp, sbuf, sdig, gofs, tn);
}

// A key array and up to three value arrays (null where a value is absent).
template <typename K, typename V0 = SortNone, typename V1 = SortNone, typename V2 = SortNone>
struct SortSet {
    K* k = nullptr;
    V0* v0 = nullptr;
    V1* v1 = nullptr;
    V2* v2 = nullptr;
};

// Runs the plan's passes: pass p reads `in` (p = 0) or the previous pass's
// output, and writes bufs[p & 1]; bufs[0] must not be `in` (bufs[1] may be:
// the first pass has consumed it before the second writes).  Returns the
// index of the buffer that holds the result.  iota: bit j set, value array j
// holds nothing yet and stands for 0, 1, ..., n - 1.  scratch: at least
// sort_scratch_bytes(n) bytes, or null to allocate it here.
template <typename K, typename V0, typename V1, typename V2>
int sort_run(const SortSet<K, V0, V1, V2>& in, const SortSet<K, V0, V1, V2> (&bufs)[2], int64_t n,
             const SortPlan& P, int iota, int* err, hipStream_t st, void* scratch, int* result) {
    *result = (P.npass - 1) & 1;
    if (n <= 0 || P.npass <= 0) return TM_OK;
    if (bufs[0].k == in.k) return tm_fail(TM_EDEVICE, "sort: the first pass would overwrite its input");
    const size_t bytes = sort_scratch_bytes(n);
    unsigned char* scr = static_cast<unsigned char*>(scratch);
    if (!scr) TM_HIP(dev_alloc((void**)&scr, bytes, st));
    uint32_t* ghist = reinterpret_cast<uint32_t*>(scr);
    uint32_t* tickets = ghist + kSortMaxPasses * kSortDigits;
    u64* status = reinterpret_cast<u64*>(scr + kSortHeadBytes);
    const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
    int rc = fill_u32(scr, (int64_t)(bytes / sizeof(uint32_t)), 0u, st);
    if (rc == TM_OK) {
        const unsigned hb = (unsigned)std::min<int64_t>(ntiles, 1024);
        hipLaunchKernelGGL((sort_hist_kernel<K>), dim3(hb), dim3(kBlock), 0, st, (const K*)in.k, n, P, ghist);
        if (hipGetLastError() != hipSuccess) rc = tm_fail(TM_EDEVICE, "sort: histogram launch");
    }
    if (rc == TM_OK) {
        hipLaunchKernelGGL(sort_base_kernel, dim3(1), dim3(kBlock), 0, st, ghist, P.npass);
        if (hipGetLastError() != hipSuccess) rc = tm_fail(TM_EDEVICE, "sort: digit start launch");
    }
    for (int p = 0; p < P.npass && rc == TM_OK; ++p) {
        const SortSet<K, V0, V1, V2>& src = p == 0 ? in : bufs[(p - 1) & 1];
        const SortSet<K, V0, V1, V2>& dst = bufs[p & 1];
        SortIO io{{src.k, src.v0, src.v1, src.v2}, {dst.k, dst.v0, dst.v1, dst.v2}};
        hipLaunchKernelGGL((sort_pass_kernel<K, V0, V1, V2>), dim3((unsigned)ntiles), dim3(kBlock), 0, st, io, n,
                           P.shift[p], P.bits[p], (uint32_t)(p + 1), p == 0 ? iota : 0,
                           (const uint32_t*)(ghist + p * kSortDigits), tickets + p, status, err);
        if (hipGetLastError() != hipSuccess) rc = tm_fail(TM_EDEVICE, "sort: pass launch");
    }
    if (!scratch) {
        const hipError_t e = dev_free(scr, st);
        if (rc == TM_OK && e != hipSuccess) rc = tm_fail(TM_EDEVICE, "sort: free");
    }
    return rc;
}

// Sorts `in` by bits [lo_bit, nbits) of its keys into `out`, stably, with
// `tmp` as the other buffer of the passes (`in` is left as it was unless
// tmp is `in`, which is allowed only when an odd number of passes runs).  At
// least one pass runs: a stable copy when no bit is sorted.
template <typename K, typename V0, typename V1, typename V2>
int sort_into(const SortSet<K, V0, V1, V2>& in, const SortSet<K, V0, V1, V2>& out,
              const SortSet<K, V0, V1, V2>& tmp, int64_t n, int lo_bit, int nbits, int iota, int* err,
              hipStream_t st) {
    SortPlan P = sort_plan(lo_bit, nbits);
    if (P.npass == 0) {
        P.npass = 1;
        P.shift[0] = 0;
        P.bits[0] = 0;
    }
    const SortSet<K, V0, V1, V2> bufs[2] = {(P.npass & 1) ? out : tmp, (P.npass & 1) ? tmp : out};
    int res = 0;
    return sort_run(in, bufs, n, P, iota, err, st, nullptr, &res);
}

// Sorts (keys, vals) by bits [lo_bit, nbits) of the key, stably.  Buffers
// ping-pong between (keys, vals) and (tkeys, tvals); on return *k_out /
// *v_out point to whichever pair holds the result (the tkeys pair after an
// odd number of passes).  iota_vals: vals holds nothing yet and stands for
// 0 .. n-1.  scratch_ext: sort_scratch_bytes(n) bytes from the caller, or
// null.  err: bit kSortStall is set if a look-back wait ran out.
template <typename K>
int radix_sort_pairs(K* keys, uint32_t* vals, K* tkeys, uint32_t* tvals, int64_t n, int lo_bit, int nbits,
                     K** k_out, uint32_t** v_out, int* err, hipStream_t st, bool iota_vals = false,
                     void* scratch_ext = nullptr) {
    *k_out = keys;
    *v_out = vals;
    if (n > 1 && nbits > lo_bit) {
        using S = SortSet<K, uint32_t>;
        S in, b0, b1;
        in.k = keys;
        in.v0 = vals;
        b0.k = tkeys;
        b0.v0 = tvals;
        b1 = in;
        const S bufs[2] = {b0, b1};
        const SortPlan P = sort_plan(lo_bit, nbits);
        int res = 0;
        TM_TRY(sort_run(in, bufs, n, P, iota_vals ? 1 : 0, err, st, scratch_ext, &res));
        *k_out = bufs[res].k;
        *v_out = bufs[res].v0;
    } else if (iota_vals) {
        TM_TRY(fill_iota_u32(vals, n, st));  // no pass ran
    }
    return TM_OK;
}
