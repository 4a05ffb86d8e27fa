/*
 * collide.hip -- collision detection between agents on a hashed uniform
 * grid (the detection module of Sec. II-A: colliding agents are marked dead
 * and excluded from the simulation).
 *
 * Two alive agents collide when |p_i - p_j|^2 < (r_i + r_j)^2, evaluated in
 * FP32 as d2 = (dx*dx + dy*dy) + dz*dz with dx = x_i - x_j and
 * rr = (r_i + r_j)^2, without contraction, so the decision is the same bit
 * for bit wherever it is taken.  All decisions of one call use the alive set
 * on entry (simultaneous events).
 *
 * Grid: cell edge h = 2.02 r_max (r_max the largest radius), so any colliding
 * pair sits in the same or an adjacent cell; cells are hashed (Teschner et
 * al. 2003) into M = 2^k >= 2N buckets.  Passes: clear, count agents per
 * bucket, exclusive scan, scatter agent ids, then each alive agent tests the
 * agents of the buckets of its 27 neighbour cells.  Ids within a bucket come
 * out in atomic order, but the result (an OR over neighbours) does not
 * depend on it.  The 1 % margin in h keeps the neighbour property exact for
 * |coordinates| < 2^16 h (about 22 km for 0.17 m radii).
 */
#include "kernels.h"

namespace potato {

namespace {

constexpr int kScanBlock = 1024;

__device__ __forceinline__ uint32_t cell_hash(int32_t ix, int32_t iy, int32_t iz, uint32_t mask) {
    return ((uint32_t)ix * 73856093u ^ (uint32_t)iy * 19349663u ^ (uint32_t)iz * 83492791u) & mask;
}

__device__ __forceinline__ void cell_of(float x, float y, float z, float inv_h, int32_t& ix, int32_t& iy,
                                        int32_t& iz) {
    ix = (int32_t)floorf(x * inv_h);
    iy = (int32_t)floorf(y * inv_h);
    iz = (int32_t)floorf(z * inv_h);
}

__global__ void __launch_bounds__(256) k_coll_clear(int32_t* count, int32_t* cursor, uint32_t m) {
    for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < m; b += gridDim.x * blockDim.x) {
        count[b] = 0;
        cursor[b] = 0;
    }
}

__global__ void __launch_bounds__(256) k_coll_count(const float* rows, int64_t ld, int64_t n, const uint8_t* alive,
                                                    float inv_h, uint32_t mask, int32_t* count, uint32_t* key) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !alive[i]) return;
    int32_t ix, iy, iz;
    cell_of(rows[i], rows[ld + i], rows[2 * ld + i], inv_h, ix, iy, iz);
    const uint32_t b = cell_hash(ix, iy, iz, mask);
    key[i] = b;
    atomicAdd(&count[b], 1);
}

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

/* One block: exclusive scan of the chunk totals (any count), in place. */
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

__global__ void __launch_bounds__(256) k_coll_scatter(int64_t n, const uint8_t* alive, const uint32_t* key,
                                                      const int32_t* start, int32_t* cursor, int32_t* ids) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !alive[i]) return;
    const uint32_t b = key[i];
    ids[start[b] + atomicAdd(&cursor[b], 1)] = (int32_t)i;
}

template <bool HET>
__global__ void __launch_bounds__(256) k_coll_query(const float* rows, int64_t ld, int64_t n, const uint8_t* type,
                                                    const float* radius, float inv_h, uint32_t mask,
                                                    const int32_t* start, const int32_t* count, const int32_t* ids,
                                                    uint8_t* alive, unsigned long long* died) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !alive[i]) return;
    const float xi = rows[i], yi = rows[ld + i], zi = rows[2 * ld + i];
    const float ri = radius[HET ? type[i] : 0];
    int32_t cx, cy, cz;
    cell_of(xi, yi, zi, inv_h, cx, cy, cz);
    bool hit = false;
    for (int dz = -1; dz <= 1 && !hit; ++dz)
        for (int dy = -1; dy <= 1 && !hit; ++dy)
            for (int dx = -1; dx <= 1 && !hit; ++dx) {
                const uint32_t b = cell_hash(cx + dx, cy + dy, cz + dz, mask);
                const int32_t s = start[b], e = s + count[b];
                for (int32_t k = s; k < e; ++k) {
                    const int32_t j = ids[k];
                    if (j == (int32_t)i) continue;
                    const float rj = radius[HET ? type[j] : 0];
                    const float ex = xi - rows[j], ey = yi - rows[ld + j], ez = zi - rows[2 * ld + j];
                    const float d2 = (ex * ex + ey * ey) + ez * ez;
                    const float rs = ri + rj;
                    if (d2 < rs * rs) { hit = true; break; }
                }
            }
    if (hit) {
        /* alive[] is not read by any query of this pass (the bucket lists
         * hold the entry alive set), so it is updated in place */
        alive[i] = 0;
        if (died) atomicAdd(died, 1ull);
    }
}

}  // namespace

uint32_t collision_buckets(int64_t n) {
    uint32_t m = 1024;
    while ((int64_t)m < 2 * n) m <<= 1;
    return m;
}

int64_t collision_workspace_bytes(int64_t n) {
    const int64_t m = collision_buckets(n);
    const int64_t chunks = (m + kScanBlock - 1) / kScanBlock;
    /* count, start, cursor [m]; key, ids [n]; chunk totals + grand total */
    return (3 * m + 2 * n + chunks + 1) * 4 + 256;
}

hipError_t launch_detect_collisions(const float* rows, int64_t ld, int64_t n, const uint8_t* type,
                                    const float* radius_dev, float r_max, uint8_t* alive,
                                    unsigned long long* died, void* workspace, hipStream_t s) {
    const uint32_t m = collision_buckets(n);
    const uint32_t chunks = (m + kScanBlock - 1) / kScanBlock;
    int32_t* count = reinterpret_cast<int32_t*>(workspace);
    int32_t* start = count + m;
    int32_t* cursor = start + m;
    uint32_t* key = reinterpret_cast<uint32_t*>(cursor + m);
    int32_t* ids = reinterpret_cast<int32_t*>(key + n);
    int32_t* totals = ids + n;
    int32_t* grand = totals + chunks;
    const float inv_h = 1.0f / (2.02f * r_max);
    const uint32_t mask = m - 1;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_coll_clear, dim3((m + 255) / 256 < 4096 ? (m + 255) / 256 : 4096), dim3(256), 0, s, count,
                       cursor, m);
    hipLaunchKernelGGL(k_coll_count, dim3(nb), dim3(256), 0, s, rows, ld, n, alive, inv_h, mask, count, key);
    hipLaunchKernelGGL(k_scan_chunks, dim3(chunks), dim3(kScanBlock), 0, s, count, start, totals, m);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanBlock), 0, s, totals, chunks, grand);
    hipLaunchKernelGGL(k_scan_add, dim3(chunks), dim3(kScanBlock), 0, s, start, totals, m);
    hipLaunchKernelGGL(k_coll_scatter, dim3(nb), dim3(256), 0, s, n, alive, key, start, cursor, ids);
    if (type)
        hipLaunchKernelGGL(k_coll_query<true>, dim3(nb), dim3(256), 0, s, rows, ld, n, type, radius_dev, inv_h,
                           mask, start, count, ids, alive, died);
    else
        hipLaunchKernelGGL(k_coll_query<false>, dim3(nb), dim3(256), 0, s, rows, ld, n, type, radius_dev, inv_h,
                           mask, start, count, ids, alive, died);
    return hipGetLastError();
}

}  // namespace potato
