/*
 * scan.h -- exclusive prefix sum of int32 counts on the device, in three
 * launches: per-chunk scans with chunk totals, one block scanning the
 * totals, and the totals added back.  Used by the collision pass (its
 * partition offsets, which add the totals where they are read) and by the
 * type order (per-block output offsets).  Each
 * translation unit that includes it gets its own copy of the kernels.
 */
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace potato {
namespace {

constexpr int kScanBlock = 1024;

/* Exclusive scan in chunks of kScanBlock: per-chunk scan + chunk totals. */
__global__ void __launch_bounds__(kScanBlock) k_scan_chunks(const int32_t* in, int32_t* out, int32_t* totals,
                                                            uint32_t m) {
    __shared__ int32_t buf[kScanBlock];
    const uint32_t g = blockIdx.x * kScanBlock + threadIdx.x;
    const int32_t v = g < m ? in[g] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        const int32_t add = (int)threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
        __syncthreads();
        buf[threadIdx.x] += add;
        __syncthreads();
    }
    if (g < m) out[g] = buf[threadIdx.x] - v;
    if (threadIdx.x == kScanBlock - 1) totals[blockIdx.x] = buf[threadIdx.x];
}

/* One block: exclusive scan of the chunk totals (any count), in place;
 * the grand total goes to *grand. */
__global__ void __launch_bounds__(kScanBlock) k_scan_totals(int32_t* totals, uint32_t n_chunks, int32_t* grand) {
    __shared__ int32_t buf[kScanBlock];
    int32_t carry = 0;
    for (uint32_t c0 = 0; c0 < n_chunks; c0 += kScanBlock) {
        const uint32_t c = c0 + threadIdx.x;
        const int32_t v = c < n_chunks ? totals[c] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kScanBlock; off <<= 1) {
            const int32_t add = (int)threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
            __syncthreads();
            buf[threadIdx.x] += add;
            __syncthreads();
        }
        if (c < n_chunks) totals[c] = carry + buf[threadIdx.x] - v;
        const int32_t chunk = buf[kScanBlock - 1];
        __syncthreads();
        carry += chunk;
    }
    if (threadIdx.x == 0) *grand = carry;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_add(int32_t* out, const int32_t* totals, uint32_t m) {
    const uint32_t g = blockIdx.x * kScanBlock + threadIdx.x;
    if (g < m) out[g] += totals[blockIdx.x];
}

/* out[0..m) = exclusive prefix sums of in[0..m); totals needs
 * scan_chunks(m) entries and *grand receives the sum of all m. */
inline uint32_t scan_chunks(uint32_t m) { return (m + kScanBlock - 1) / kScanBlock; }

inline void launch_exclusive_scan(const int32_t* in, int32_t* out, int32_t* totals, int32_t* grand, uint32_t m,
                                  hipStream_t s) {
    const uint32_t chunks = scan_chunks(m);
    hipLaunchKernelGGL(k_scan_chunks, dim3(chunks), dim3(kScanBlock), 0, s, in, out, totals, m);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanBlock), 0, s, totals, chunks, grand);
    hipLaunchKernelGGL(k_scan_add, dim3(chunks), dim3(kScanBlock), 0, s, out, totals, m);
}

/* The same without the last launch: the prefix sum of element i is
 * out[i] + totals[i / kScanBlock], added by the consumer. */
inline void launch_exclusive_scan_chunks(const int32_t* in, int32_t* out, int32_t* totals, int32_t* grand,
                                         uint32_t m, hipStream_t s) {
    const uint32_t chunks = scan_chunks(m);
    hipLaunchKernelGGL(k_scan_chunks, dim3(chunks), dim3(kScanBlock), 0, s, in, out, totals, m);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanBlock), 0, s, totals, chunks, grand);
}

}  // namespace
}  // namespace potato
