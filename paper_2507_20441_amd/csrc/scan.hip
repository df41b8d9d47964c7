// Scan of tile sums for the device-wide exclusive scan, and the digit starts
// of the radix sort (tm_primitives.h).
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

__global__ void __launch_bounds__(kBlock) sort_base_kernel(uint32_t* ghist, int npass) {
    __shared__ uint32_t wsum[kWaves];
    for (int p = 0; p < npass; ++p) {
        uint32_t* h = ghist + p * kSortDigits;
        const uint32_t v = h[threadIdx.x];
        h[threadIdx.x] = block_excl_scan_256(v, wsum);
    }
}
