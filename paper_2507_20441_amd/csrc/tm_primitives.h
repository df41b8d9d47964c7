// Device-wide primitives of the TIMEST GPU library: exclusive prefix sums and
// a stable LSD radix sort of (key, value) pairs.  Templates, instantiated by
// the translation units that use them.
#pragma once

#include "tm_internal.h"

constexpr int kScanItems = 8;                      // values per lane in a scan tile
constexpr int kScanTile = kBlock * kScanItems;     // 2048
constexpr int kSortItems = 8;                      // keys per lane in a sort tile
constexpr int kSortTile = kBlock * kSortItems;     // 2048
constexpr int kRadixMaxBits = 9;                   // sort digits: up to 9 bits, two per thread
constexpr int kRadixMax = 1 << kRadixMaxBits;

// Radix passes over nb key bits (digits of at most kRadixMaxBits, split as
// evenly as possible).
inline int radix_passes(int nb) { return nb <= 0 ? 0 : (nb + kRadixMaxBits - 1) / kRadixMaxBits; }

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
// Stable LSD radix sort of (key, value) pairs (fewer than 2^32), digits of up
// to 9 bits.
// Per pass: tile histograms (digit-major), an exclusive scan of each digit's
// row with the digit totals, then a scatter in which every wave ranks its
// keys in input order with ballots and each digit's start is the scan of the
// totals.
// ---------------------------------------------------------------------------
template <typename K>
__global__ void __launch_bounds__(kBlock)
radix_hist_kernel(const K* keys, int64_t n, int shift, int bits, uint32_t* hist, int64_t ntiles) {
    __shared__ uint32_t h[kRadixMax];
    h[threadIdx.x] = 0;
    h[threadIdx.x + kBlock] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const K mask = (K)((1u << bits) - 1);
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(uint32_t)((keys[i] >> shift) & mask)], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < (1 << bits); d += kBlock) hist[(int64_t)d * ntiles + blockIdx.x] = h[d];
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

// Per digit d < ndig: the exclusive scan of the digit's row of tile counts
// (hist[d * ntiles + tile]), in place, and the row's total in totals[d].
int radix_rowscan(uint32_t* hist, int64_t ntiles, uint32_t* totals, hipStream_t st, int ndig);

template <typename K>
__global__ void __launch_bounds__(kBlock)
radix_scatter_kernel(const K* keys, const uint32_t* vals, K* okeys, uint32_t* ovals, int64_t n,
                     int shift, int bits, const uint32_t* offs, const uint32_t* totals, int64_t ntiles, int iota) {
    static_assert(2 * kBlock == kRadixMax, "two digits per thread");
    __shared__ uint32_t cnt[kWaves][kRadixMax];
    __shared__ uint32_t dstart[kRadixMax];  // tile-local start of each digit's run
    __shared__ uint32_t gbase[kRadixMax];   // global start of this tile's run of each digit
    __shared__ K skey[kSortTile];
    __shared__ uint32_t sval[kSortTile];
    __shared__ uint32_t wsum[kWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int w = 0; w < kWaves; ++w) {
        cnt[w][threadIdx.x] = 0;
        cnt[w][threadIdx.x + kBlock] = 0;
    }
    __syncthreads();
    const K mask = (K)((1u << bits) - 1);
    const u64 lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    // wave w owns tile positions [w*64*kSortItems, (w+1)*64*kSortItems), in
    // rounds of 64 consecutive keys: the wave sees its keys in input order
    const int64_t tbase = (int64_t)blockIdx.x * kSortTile;
    const int64_t wbase = tbase + (int64_t)wave * 64 * kSortItems;
    K key[kSortItems];
    uint32_t val[kSortItems];
    uint32_t dig[kSortItems];
    uint32_t rank[kSortItems];
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t i = wbase + (int64_t)k * 64 + lane;
        const bool ok = i < n;
        key[k] = ok ? keys[i] : (K)0;
        val[k] = ok ? (iota ? (uint32_t)i : vals[i]) : 0u;
        const uint32_t d = ok ? (uint32_t)((key[k] >> shift) & mask) : 0u;
        dig[k] = d;
        u64 peers = __ballot(ok);
        for (int b = 0; b < bits; ++b) {
            const u64 bal = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t before = cnt[wave][d];
        rank[k] = before + (uint32_t)__popcll(peers & lt_mask);
        // the lowest lane of each digit group advances the wave's counter
        if (ok && (peers & lt_mask) == 0) cnt[wave][d] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per digit pair (d0, d1 = 2t, 2t + 1 for thread t, so that scans over the
    // threads run in digit order): the tile's counts, their exclusive scan
    // over digits (the tile-local start), and each wave's start inside it
    const int ndig = 1 << bits;
    const uint32_t d0 = 2 * threadIdx.x, d1 = d0 + 1;
    uint32_t t0 = 0, t1 = 0;
    for (int w = 0; w < kWaves; ++w) {
        t0 += cnt[w][d0];
        t1 += cnt[w][d1];
    }
    // global start of this tile's run of a digit: the digit's start (scan of
    // the digit totals) plus the earlier tiles' counts of it
    const uint32_t g0 = (int)d0 < ndig ? totals[d0] : 0u, g1 = (int)d1 < ndig ? totals[d1] : 0u;
    const uint32_t gb = block_excl_scan_256(g0 + g1, wsum);
    if ((int)d0 < ndig) gbase[d0] = gb + offs[(int64_t)d0 * ntiles + blockIdx.x];
    if ((int)d1 < ndig) gbase[d1] = gb + g0 + offs[(int64_t)d1 * ntiles + blockIdx.x];
    const uint32_t local = block_excl_scan_256(t0 + t1, wsum);
    {
        uint32_t run0 = local, run1 = local + t0;  // exclusive
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t c0 = cnt[w][d0], c1 = cnt[w][d1];
            cnt[w][d0] = run0;
            cnt[w][d1] = run1;
            run0 += c0;
            run1 += c1;
        }
    }
    __syncthreads();
    dstart[d0] = cnt[0][d0];
    dstart[d1] = cnt[0][d1];
    // keys to their tile-local sorted places
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t i = wbase + (int64_t)k * 64 + lane;
        if (i < n) {
            const uint32_t lp = cnt[wave][dig[k]] + rank[k];
            skey[lp] = key[k];
            sval[lp] = val[k];
        }
    }
    __syncthreads();
    // out in tile-local order: each digit's run goes to consecutive addresses
    const int tn = (int)((n - tbase) < kSortTile ? (n - tbase) : kSortTile);
    for (int p = threadIdx.x; p < tn; p += kBlock) {
        const K kk = skey[p];
        const uint32_t dd = (uint32_t)((kk >> shift) & mask);
        const uint32_t gpos = gbase[dd] + ((uint32_t)p - dstart[dd]);
        okeys[gpos] = kk;
        ovals[gpos] = sval[p];
    }
}

struct HistReader {
    const uint32_t* h;
    __device__ uint32_t operator()(int64_t i) const { return h[i]; }
};

// Sorts (keys, vals) by bits [lo_bit, nbits) of the key, stably.  Buffers
// ping-pong between (keys, vals) and (tkeys, tvals); on return *k_out / *v_out
// point to whichever pair holds the result.  iota_vals: vals holds nothing
// yet and stands for 0 .. n-1 (the first pass makes them).
template <typename K>
int radix_sort_pairs(K* keys, uint32_t* vals, K* tkeys, uint32_t* tvals, int64_t n, int lo_bit,
                     int nbits, K** k_out, uint32_t** v_out, int* ovf, hipStream_t st, bool iota_vals = false,
                     uint32_t* hist_ext = nullptr) {
    K* ka = keys;
    uint32_t* va = vals;
    K* kb = tkeys;
    uint32_t* vb = tvals;
    if (n > 1 && nbits > lo_bit) {
        const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
        const int npass = radix_passes(nbits - lo_bit);
        const int64_t maxdig = (int64_t)1 << ((nbits - lo_bit + npass - 1) / npass);
        // the digit histograms: (ntiles + 1) * maxdig words, from the caller
        // (hist_ext, which must hold that many) or allocated here
        uint32_t* hist = hist_ext;
        if (!hist) TM_HIP(dev_alloc((void**)&hist, (ntiles * maxdig + maxdig) * sizeof(uint32_t), st));
        uint32_t* totals = hist + ntiles * maxdig;
        int shift = lo_bit;
        for (int p = 0; p < npass; ++p) {
            const int bits = (nbits - shift + (npass - p) - 1) / (npass - p);
            hipLaunchKernelGGL((radix_hist_kernel<K>), dim3((unsigned)ntiles), dim3(kBlock), 0, st,
                               (const K*)ka, n, shift, bits, hist, ntiles);
            TM_HIP(hipGetLastError());
            TM_TRY(radix_rowscan(hist, ntiles, totals, st, 1 << bits));
            hipLaunchKernelGGL((radix_scatter_kernel<K>), dim3((unsigned)ntiles), dim3(kBlock), 0,
                               st, (const K*)ka, (const uint32_t*)va, kb, vb, n, shift, bits,
                               (const uint32_t*)hist, (const uint32_t*)totals, ntiles, (iota_vals && p == 0) ? 1 : 0);
            TM_HIP(hipGetLastError());
            K* tk = ka; ka = kb; kb = tk;
            uint32_t* tv = va; va = vb; vb = tv;
            shift += bits;
        }
        if (!hist_ext) TM_HIP(dev_free(hist, st));
    }
    if (iota_vals && !(n > 1 && nbits > lo_bit)) TM_TRY(fill_iota_u32(va, n, st));  // no pass ran
    *k_out = ka;
    *v_out = va;
    return TM_OK;
}
