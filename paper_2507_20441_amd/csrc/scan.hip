// Scan of tile sums for the device-wide exclusive scan, and the per-digit row
// scans of the radix sort (tm_primitives.h).
#include <algorithm>

#include "tm_primitives.h"

namespace {

// One block scans up to kScanTile values in place: a[0..n] (a[n] = total).
__global__ void __launch_bounds__(kBlock) scan_single_kernel(u128* a, int64_t n, int* ovf) {
    const int64_t first = (int64_t)threadIdx.x * kScanItems;
    u128 v[kScanItems];
    u128 s = 0;
    bool carry = false;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = first + k;
        v[k] = i < n ? a[i] : (u128)0;
        u128 y = s + v[k];
        if (y < s) carry = true;
        s = y;
    }
    u128 tot;
    u128 run = block_exclusive(s, &tot, &carry);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = first + k;
        if (i < n) a[i] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) a[n] = tot;
    if (carry) atomicOr(ovf, 1);
}

// One block per digit; each lane owns a run of consecutive tiles.  Rows of
// up to kRowLds tiles go through LDS, so that the row is read and written
// with consecutive addresses.
constexpr int kRowLds = 8192;

__global__ void __launch_bounds__(kBlock) radix_rowscan_kernel(uint32_t* hist, int64_t ntiles, uint32_t* totals) {
    __shared__ uint32_t wsum[kWaves];
    __shared__ uint32_t buf[kRowLds];
    uint32_t* row = hist + (int64_t)blockIdx.x * ntiles;
    const bool staged = ntiles <= kRowLds;
    uint32_t* r = staged ? buf : row;
    if (staged) {
        for (int64_t i = threadIdx.x; i < ntiles; i += kBlock) buf[i] = row[i];
        __syncthreads();
    }
    const int64_t per = (ntiles + kBlock - 1) / kBlock;
    const int64_t lo = (int64_t)threadIdx.x * per;
    const int64_t hi = lo + per < ntiles ? lo + per : ntiles;
    uint32_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += r[i];
    uint32_t run = block_excl_scan_256(s, wsum);
    for (int64_t i = lo; i < hi; ++i) {
        const uint32_t c = r[i];
        r[i] = run;
        run += c;
    }
    if (threadIdx.x == kBlock - 1) totals[blockIdx.x] = run;
    if (staged) {
        __syncthreads();
        for (int64_t i = threadIdx.x; i < ntiles; i += kBlock) row[i] = buf[i];
    }
}

}  // namespace

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        p[i] = v;
}

int fill_u32(void* p, int64_t n_words, uint32_t v, hipStream_t st) {
    if (n_words <= 0) return TM_OK;
    const int64_t blocks = std::min<int64_t>((n_words + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st,
                       static_cast<uint32_t*>(p), n_words, v);
    TM_HIP(hipGetLastError());
    return TM_OK;
}

__global__ void fill_iota_kernel(uint32_t* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        p[i] = (uint32_t)i;
}

int fill_iota_u32(uint32_t* p, int64_t n, hipStream_t st) {
    if (n <= 0) return TM_OK;
    const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(fill_iota_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st, p, n);
    TM_HIP(hipGetLastError());
    return TM_OK;
}

int scan_parts(u128* part, int64_t nb, int* ovf, hipStream_t st) {
    if (nb <= kScanTile) {
        hipLaunchKernelGGL(scan_single_kernel, dim3(1), dim3(kBlock), 0, st, part, nb, ovf);
        TM_HIP(hipGetLastError());
        return TM_OK;
    }
    return device_exclusive_scan<u128>(ArrayReader128{part}, nb, part, ovf, st);
}

int radix_rowscan(uint32_t* hist, int64_t ntiles, uint32_t* totals, hipStream_t st, int ndig) {
    hipLaunchKernelGGL(radix_rowscan_kernel, dim3((unsigned)ndig), dim3(kBlock), 0, st, hist, ntiles, totals);
    TM_HIP(hipGetLastError());
    return TM_OK;
}
