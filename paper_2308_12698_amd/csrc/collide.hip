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
 * pair sits in the same or an adjacent cell; cells map to M = 2^k >= 2N
 * buckets by the low bits of their Z-order (Morton) code.  Passes: clear, count agents per
 * bucket, exclusive scan, counting-sort scatter of (id, x, y, z, radius)
 * into bucket order, then one thread per sorted slot tests the slots of the
 * buckets of its 27 neighbour cells.  Slots within a bucket come out in
 * atomic order, but the result (an OR over neighbours) does not depend on
 * it.  The 1 % margin in h keeps the neighbour property exact for
 * |coordinates| < 2^16 h (about 22 km for 0.17 m radii).
 */
#include <mutex>
#include <vector>

#include "kernels.h"
#include "scan.h"

namespace potato {

/* Cells whose first two candidates are loaded together in the query (a
 * divisor of 27).  At 1M agents a pass took 0.36 ms with 3, 0.37 with 1
 * and with 9 (150 VGPRs), 0.48 with 27 (more registers than two waves per
 * SIMD allow). */
#ifndef POTATO_QUERY_CELLS_PER_GROUP
#define POTATO_QUERY_CELLS_PER_GROUP 3
#endif

namespace {


/* Low 10 bits of v moved to every third bit position (bit interleaving for
 * a Morton / Z-order code). */
__device__ __forceinline__ uint32_t spread3(int32_t v) {
    uint32_t x = (uint32_t)v & 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

/* Bucket of a cell: the low bits of its Z-order code, i.e. a grid that wraps
 * around every 2^(bits/3) cells per axis.  Cells that share a bucket are far
 * apart and fail the distance test; cells that are close get nearby bucket
 * numbers, so agents sorted by bucket are sorted along a space-filling
 * curve and neighbouring threads of the query read the same buckets. */
__device__ __forceinline__ uint32_t cell_bucket(uint32_t sx, uint32_t sy, uint32_t sz, uint32_t mask) {
    return (sx | (sy << 1) | (sz << 2)) & mask;
}

/* Cell index along one axis.  The coordinate in cells is clamped to
 * [-2^24, 2^24] before the conversion, so infinite, NaN (max/min return the
 * other operand) and huge coordinates give a defined index and the
 * neighbour indices +-1 cannot overflow.  Agents beyond the clamp share the
 * edge cells, which only adds candidates; the decision is the distance
 * test, and a NaN or infinite position never passes it. */
__device__ __forceinline__ int32_t cell_index(float x, float inv_h) {
    const float c = fminf(fmaxf(x * inv_h, -16777216.0f), 16777216.0f);
    return (int32_t)floorf(c);
}

__device__ __forceinline__ void cell_of(float x, float y, float z, float inv_h, int32_t& ix, int32_t& iy,
                                        int32_t& iz) {
    ix = cell_index(x, inv_h);
    iy = cell_index(y, inv_h);
    iz = cell_index(z, inv_h);
}

__global__ void __launch_bounds__(256) k_coll_clear(int32_t* count, uint32_t m) {
    for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < m; b += gridDim.x * blockDim.x) count[b] = 0;
}

__global__ void __launch_bounds__(256) k_coll_count(const float* rows, int64_t ld, int64_t n, const uint8_t* alive,
                                                    float inv_h, uint32_t mask, int32_t* count, uint32_t* key) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !alive[i]) return;
    int32_t ix, iy, iz;
    cell_of(rows[i], rows[ld + i], rows[2 * ld + i], inv_h, ix, iy, iz);
    const uint32_t b = cell_bucket(spread3(ix), spread3(iy), spread3(iz), mask);
    key[i] = b;
    atomicAdd(&count[b], 1);
}

/* Counting sort of the alive agents by bucket: agent i gets a slot in its
 * bucket's range (taking the bucket's count down to zero), and the slot
 * receives the agent id and (x, y, z, radius), so that the query reads each
 * bucket's candidates from consecutive addresses. */
__global__ void __launch_bounds__(256) k_coll_scatter(const float* rows, int64_t ld, int64_t n, const uint8_t* alive,
                                                      const uint8_t* type, int n_types, const float* radius,
                                                      const uint32_t* key,
                                                      const int32_t* start, int32_t* count, int32_t* ids,
                                                      float4* spos) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !alive[i]) return;
    const uint32_t b = key[i];
    const int32_t slot = start[b] + atomicSub(&count[b], 1) - 1;
    ids[slot] = (int32_t)i;
    spos[slot] = make_float4(rows[i], rows[ld + i], rows[2 * ld + i],
                             radius[type ? type_entry(type, (uint32_t)i, n_types) : 0]);
}

/* One thread per sorted slot: consecutive lanes hold agents of the same or
 * nearby cells, so the bucket ranges and candidate positions they read are
 * shared through the caches. */
__global__ void __launch_bounds__(256) k_coll_query(const float4* spos, const int32_t* ids, const int32_t* start,
                                                    const int32_t* total, float inv_h, uint32_t mask,
                                                    uint8_t* alive, unsigned long long* died) {
#pragma clang fp contract(off)
    const int32_t k = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= *total) return;
    const float4 pk = spos[k];
    int32_t cx, cy, cz;
    cell_of(pk.x, pk.y, pk.z, inv_h, cx, cy, cz);
    const uint32_t sx[3] = {spread3(cx - 1), spread3(cx), spread3(cx + 1)};
    const uint32_t sy[3] = {spread3(cy - 1), spread3(cy), spread3(cy + 1)};
    const uint32_t sz[3] = {spread3(cz - 1), spread3(cz), spread3(cz + 1)};
    /* all 27 bucket ranges are requested before any is used, so their
     * loads are in flight together instead of one round trip per cell */
    int32_t lo[27], hi[27];
#pragma unroll
    for (int c = 0; c < 27; ++c) {
        const uint32_t b = cell_bucket(sx[c % 3], sy[(c / 3) % 3], sz[c / 9], mask);
        lo[c] = start[b];
        hi[c] = start[b + 1];
    }
    /* The decision for one candidate j: the same FP32 operations, in the
     * same order, as the reference's pair test. */
    auto collides = [&](const float4& pj) {
        const float ex = pk.x - pj.x, ey = pk.y - pj.y, ez = pk.z - pj.z;
        const float d2 = (ex * ex + ey * ey) + ez * ez;
        const float rs = pk.w + pj.w;
        return d2 < rs * rs;
    };
    /* Candidates are read in groups of three cells, the first two slots of
     * each cell unconditionally (at a clamped, always valid index, the
     * result masked), so that six independent loads are in flight per
     * round trip instead of one load per dependent loop iteration; a cell
     * holds ~0.5 candidates on average, and the rare further ones are read
     * by a loop. */
    const int32_t last = *total - 1;
    bool hit = false;
    constexpr int G = POTATO_QUERY_CELLS_PER_GROUP;
#pragma unroll
    for (int g = 0; g < 27 / G; ++g) {
        float4 pc[2 * G];
        bool use[2 * G];
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int c = G * g + u;
            const int32_t j0 = lo[c], j1 = lo[c] + 1;
            pc[2 * u] = spos[j0 < last ? j0 : last];
            pc[2 * u + 1] = spos[j1 < last ? j1 : last];
            use[2 * u] = j0 < hi[c] && j0 != k;
            use[2 * u + 1] = j1 < hi[c] && j1 != k;
        }
#pragma unroll
        for (int t = 0; t < 2 * G; ++t) hit |= use[t] && collides(pc[t]);
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int c = G * g + u;
            for (int32_t j = lo[c] + 2; j < hi[c]; ++j)
                if (j != k) hit |= collides(spos[j]);
        }
    }
    /* the query reads positions from the sorted copy only, so the mask is
     * updated in place */
    if (hit) alive[ids[k]] = 0;
    if (died) {
        /* one atomic per wave: most agents of a dense swarm collide, and one
         * atomic each on a single counter serialises the whole pass */
        const unsigned long long m = __ballot(hit);
        if (m && (threadIdx.x & (warpSize - 1)) == (unsigned)(__ffsll((long long)m) - 1))
            atomicAdd(died, (unsigned long long)__popcll(m));
    }
}

}  // namespace

/* Buckets per agent (rounded up to a power of two).  More buckets mean
 * fewer far cells sharing a bucket, but longer clear and scan passes: at
 * 1M agents 2 measured 0.36 ms per pass, 4, 8 and 16 0.37, 0.40, 0.47. */
#ifndef POTATO_BUCKETS_PER_AGENT
#define POTATO_BUCKETS_PER_AGENT 2
#endif

namespace {

constexpr uint32_t buckets_for(int64_t n) {
    uint32_t m = 1024;
    while ((int64_t)m < POTATO_BUCKETS_PER_AGENT * n && m < (1u << 30)) m <<= 1;   /* the Z-order code has 30 bits */
    return m;
}

constexpr int64_t workspace_for(int64_t n) {
    const int64_t m = buckets_for(n);
    const int64_t chunks = (m + kScanBlock - 1) / kScanBlock;
    /* sorted (x, y, z, r) [n] first (16-byte aligned); count [m]; start [m+1];
     * key, ids [n]; chunk totals [chunks] */
    return 16 * n + (m + (m + 1) + 2 * n + chunks) * 4 + 256;
}

/* Workspace of the allocation-free entry point: a file-scope device array
 * sized for the largest swarm it accepts.  Every GPU the library runs on
 * holds its own copy until the process ends; host code reaches it only
 * through the address hipGetSymbolAddress returns for the current device
 * (the array's name in host code is not a device address). */
constexpr int64_t kNoAllocBytes = workspace_for(kNoAllocMaxAgents);

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

uint32_t collision_buckets(int64_t n) { return buckets_for(n); }

int64_t collision_workspace_bytes(int64_t n) { return workspace_for(n); }

hipError_t collision_scratch(void** ptr, int64_t* bytes) {
    static std::mutex mu;
    static std::vector<void*> addr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> g(mu);
    if ((size_t)dev >= addr.size()) addr.resize((size_t)dev + 1, nullptr);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = kNoAllocBytes;
    return hipSuccess;
}

hipError_t launch_detect_collisions(const float* rows, int64_t ld, int64_t n, const uint8_t* type, int n_types,
                                    const float* radius_dev, float r_max, uint8_t* alive,
                                    unsigned long long* died, void* workspace, hipStream_t s) {
    const uint32_t m = collision_buckets(n);
    float4* spos = reinterpret_cast<float4*>(workspace);
    int32_t* count = reinterpret_cast<int32_t*>(spos + n);
    int32_t* start = count + m;
    uint32_t* key = reinterpret_cast<uint32_t*>(start + m + 1);
    int32_t* ids = reinterpret_cast<int32_t*>(key + n);
    int32_t* totals = ids + n;
    const float inv_h = 1.0f / (2.02f * r_max);
    const uint32_t mask = m - 1;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_coll_clear, dim3((m + 255) / 256 < 4096 ? (m + 255) / 256 : 4096), dim3(256), 0, s, count, m);
    hipLaunchKernelGGL(k_coll_count, dim3(nb), dim3(256), 0, s, rows, ld, n, alive, inv_h, mask, count, key);
    launch_exclusive_scan(count, start, totals, start + m, m, s);   /* grand total in start[m] */
    hipLaunchKernelGGL(k_coll_scatter, dim3(nb), dim3(256), 0, s, rows, ld, n, alive, type, n_types, radius_dev, key,
                       start, count, ids, spos);
    hipLaunchKernelGGL(k_coll_query, dim3(nb), dim3(256), 0, s, spos, ids, start, start + m, inv_h, mask, alive,
                       died);
    return hipGetLastError();
}

}  // namespace potato
