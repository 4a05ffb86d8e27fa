/*
 * collide.hip -- collision detection between agents on a wrapped uniform
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
 * pair sits in the same or an adjacent cell.  Cells map to buckets by their
 * indices wrapped to 2^bx x 2^by x 2^bz, where the bits split the budget
 * 2^k >= 2N by the extent of the alive agents' bounding box (so a flat
 * swarm does not leave the buckets of an unused depth empty); buckets are
 * linear with x fastest, and each x row holds two extra ghost columns (a
 * copy of the last column before the first and of the first after the
 * last), so the three x neighbours of any cell are three consecutive
 * buckets and a cell's 27 neighbours are 9 contiguous bucket ranges.
 * Passes: bounding box (block partials, reduced again by every block of
 * the next kernel); a two-level sort of (x, y, z, radius) and the agent id
 * into bucket order (per-tile counts of bucket partitions, their scan, the
 * tiles' items written partition by partition, then each window of a
 * partition sorted in LDS, which also writes the bucket starts); query, one
 * thread per sorted slot, over the candidates of its 9 ranges in batches of
 * loads in flight; one block adding up the dead.  Cells that share a bucket
 * are far apart and fail the distance test; the decision is always the
 * distance test.  The 1 % margin in h keeps
 * the neighbour property exact for |coordinates| < 2^16 h (about 22 km for
 * 0.17 m radii).
 */
#include <mutex>
#include <vector>

#include "kernels.h"
#include "scan.h"

namespace potato {

/* Candidates whose loads are issued together in the query. */
#ifndef POTATO_QUERY_BATCH
#define POTATO_QUERY_BATCH 8
#endif

namespace {

/* Fewest bits of the ghost-padded x axis: 2^5 columns + 2 ghosts keeps the
 * padding within 1/16 of the bucket budget. */
constexpr int kMinXBits = 5;

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

/* Wrap of the grid: 2^bx x 2^by x 2^bz cells, x rows of 2^bx + 2 buckets. */
struct Wrap {
    int bx, by, bz;
    uint32_t mx, my, mz;     /* 2^b - 1 */
    uint32_t row;            /* 2^bx + 2 */
};

__device__ __forceinline__ int ceil_log2(int64_t e) {
    int b = 0;
    while (b < 40 && (int64_t(1) << b) < e) ++b;
    return b;
}

/* Bits per axis for bucket budget 2^k from the bounding box (min x, y, z,
 * max x, y, z, in cells): start from the bits that cover each extent, then
 * take bits away, each time from the axis whose extent is the smallest
 * multiple of its halved wrap (it gains the fewest wraps), x not below
 * kMinXBits.  Wave-uniform: every kernel of a pass computes the same wrap. */
__device__ __forceinline__ Wrap plan_wrap(const int32_t* box, int k) {
    int64_t e[3];
    for (int a = 0; a < 3; ++a) {
        const int64_t lo = box[a], hi = box[3 + a];
        e[a] = hi >= lo ? hi - lo + 1 : 1;       /* no alive agent: any wrap */
    }
    int b[3] = {ceil_log2(e[0]), ceil_log2(e[1]), ceil_log2(e[2])};
    if (b[0] < kMinXBits) b[0] = kMinXBits;
    while (b[0] + b[1] + b[2] > k) {
        int best = -1;
        for (int a = 2; a >= 0; --a) {
            if (b[a] == 0 || (a == 0 && b[a] == kMinXBits)) continue;
            /* e[a] / 2^(b[a]-1) < e[best] / 2^(b[best]-1), cross-multiplied */
            if (best < 0 || e[a] * (int64_t(1) << b[best]) < e[best] * (int64_t(1) << b[a])) best = a;
        }
        --b[best];
    }
    Wrap w;
    w.bx = b[0]; w.by = b[1]; w.bz = b[2];
    w.mx = (1u << b[0]) - 1u; w.my = (1u << b[1]) - 1u; w.mz = (1u << b[2]) - 1u;
    w.row = (1u << b[0]) + 2u;
    return w;
}

/* Bucket of wrapped cell (column col = wrapped x + 1, wrapped y, wrapped z). */
__device__ __forceinline__ uint32_t bucket_of(const Wrap& w, uint32_t col, uint32_t wy, uint32_t wz) {
    return col + w.row * (wy | (wz << w.by));
}

/* Bounding box of the alive agents' cells, in two steps: each block of a
 * grid of at most kBoxBlocks reduces its grid-stride share to six partial
 * bounds, then every block of the next kernel reduces the partials itself
 * (one atomic per block on six shared words serialised the first form of
 * this pass: 96 us at 1M agents). */
constexpr int kBoxBlocks = 1024;
constexpr int kMaxWaves = 16;

__device__ __forceinline__ int32_t bound_op(int a, int32_t x, int32_t y) { return a < 3 ? min(x, y) : max(x, y); }

/* Block reduction of v[6] (min of 0-2, max of 3-5); the result is valid in
 * thread 0..5 as red[a][0]. */
__device__ __forceinline__ void block_bounds(int32_t v[6], int32_t (*red)[kMaxWaves]) {
    for (int a = 0; a < 6; ++a) {
        int32_t x = v[a];
        for (int off = 32; off > 0; off >>= 1) x = bound_op(a, x, __shfl_xor(x, off));
        v[a] = x;
    }
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < 6; ++a) red[a][threadIdx.x / 64] = v[a];
    __syncthreads();
    if (threadIdx.x < 6) {
        const int a = threadIdx.x;
        int32_t x = red[a][0];
        for (int w = 1; w < (int)(blockDim.x / 64); ++w) x = bound_op(a, x, red[a][w]);
        red[a][0] = x;
    }
}

__global__ void __launch_bounds__(256) k_coll_bounds(const float* rows, int64_t ld, int64_t n, const uint8_t* alive,
                                                     float inv_h, int32_t* partial) {
    __shared__ int32_t red[6][kMaxWaves];
    int32_t v[6] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MIN, INT32_MIN, INT32_MIN};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (!alive[i]) continue;
        for (int a = 0; a < 3; ++a) {
            const int32_t c = cell_index(rows[a * ld + i], inv_h);
            v[a] = min(v[a], c);
            v[3 + a] = max(v[3 + a], c);
        }
    }
    block_bounds(v, red);
    if (threadIdx.x < 6) partial[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

/* The bounding box from the partials of k_coll_bounds, in every thread of
 * the block (box_lds: six words of LDS). */
__device__ __forceinline__ void reduce_box(const int32_t* partial, int n_partial, int32_t (*red)[kMaxWaves],
                                           int32_t* box_lds) {
    int32_t v[6] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MIN, INT32_MIN, INT32_MIN};
    for (int b = threadIdx.x; b < n_partial; b += blockDim.x)
        for (int a = 0; a < 6; ++a) v[a] = bound_op(a, v[a], partial[b * 6 + a]);
    block_bounds(v, red);
    if (threadIdx.x < 6) box_lds[threadIdx.x] = red[threadIdx.x][0];
    __syncthreads();
}

/* Blocks are dispatched to the 8 XCDs in turn (block b to XCD b mod 8), and
 * each XCD has its own L2.  Mapping block b to tile xcd * (blocks per XCD) +
 * b / 8 gives each XCD one contiguous eighth of the tiles, so neighbouring
 * tiles, which read the same data, share an L2. */
constexpr uint32_t kXcds = 8;

__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n_blocks) {
    const uint32_t q = n_blocks / kXcds, r = n_blocks % kXcds;
    const uint32_t x = b % kXcds, pos = b / kXcds;
    return x * q + (x < r ? x : r) + pos;
}

/* Wrapped cell of a position. */
__device__ __forceinline__ void wrapped_cell(const Wrap& w, float x, float y, float z, float inv_h, uint32_t& wx,
                                             uint32_t& wy, uint32_t& wz) {
    wx = (uint32_t)cell_index(x, inv_h) & w.mx;
    wy = (uint32_t)cell_index(y, inv_h) & w.my;
    wz = (uint32_t)cell_index(z, inv_h) & w.mz;
}

/* An agent in the first wrapped column also sits in the ghost column after
 * the last, one in the last column in the ghost column before the first:
 * the bucket offset of its ghost, or 0. */
__device__ __forceinline__ int32_t ghost_offset(const Wrap& w, uint32_t wx) {
    return wx == 0 ? (int32_t)(w.mx + 1) : (wx == w.mx ? -(int32_t)(w.mx + 1) : 0);
}

/* Bucket of an item: the agent's own bucket, or for a ghost copy (id with
 * the top bit set) the ghost bucket of its edge column. */
__device__ __forceinline__ uint32_t item_bucket(const Wrap& w, const float4& q, int32_t id, float inv_h) {
    uint32_t wx, wy, wz;
    wrapped_cell(w, q.x, q.y, q.z, inv_h, wx, wy, wz);
    const uint32_t b = bucket_of(w, wx + 1, wy, wz);
    return id < 0 ? (uint32_t)((int32_t)b + ghost_offset(w, wx)) : b;
}

/* Sort of the items into bucket order.  An item is an alive agent, or the
 * ghost copy of an agent in an edge column.  Two levels:
 *  - the buckets are split into partitions of 2^s consecutive buckets (s the
 *    smallest >= kWindowBits that gives at most kMaxParts partitions) and
 *    the agents into tiles (tiles of one XCD contiguous, as in xcd_tile).
 *    k_coll_hist counts each tile's items per partition in LDS; one
 *    exclusive scan over the counts, laid out partition-major, gives every
 *    (partition, tile) pair its output offset; k_coll_part writes each
 *    tile's items through LDS cursors.  The tiles of one XCD thus write one
 *    contiguous run per partition, which its L2 merges into whole lines.
 *  - k_coll_sort, one block per window of kWindow buckets, counts in LDS the
 *    items of its partition that fall in its window (and those of the
 *    partition's earlier windows), scans the counts into the window's
 *    bucket starts, and places its items within the partition's range.
 * The order of the items of one bucket follows the order of the LDS
 * atomics; no decision of the query depends on it. */
constexpr int kWindowBits = 12;
constexpr int kWindow = 1 << kWindowBits;
constexpr int64_t kMaxParts = 16384;        /* LDS cursors of the tile passes: 64 KB */
constexpr int kTileBlock = 512;
constexpr int kTileUnroll = 4;
constexpr int64_t kTileAgents = kTileBlock * kTileUnroll;
constexpr int64_t kMaxTiles = 2048;

/* Offset of (partition, tile) cell c after the scan in chunks: the chunk's
 * own exclusive scan plus the scanned chunk totals; cell `cells` holds the
 * slot count. */
__device__ __forceinline__ int32_t cell_offset(const int32_t* off, const int32_t* totals, int64_t c, int64_t cells) {
    return c < cells ? off[c] + totals[c / kScanBlock] : off[cells];
}

/* Also reduces the bounding box: block 0 stores it for the later kernels
 * of the pass. */
__global__ void __launch_bounds__(kTileBlock) k_coll_hist(const float* rows, int64_t ld, int64_t n,
                                                          const uint8_t* alive, float inv_h, const int32_t* partial,
                                                          int n_partial, int32_t* box, int k,
                                                          int s, int32_t parts, int64_t tile, int32_t* hist) {
    extern __shared__ int32_t cnt[];
    __shared__ int32_t red[6][kMaxWaves];
    __shared__ int32_t box_lds[6];
    const uint32_t t = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t a0 = (int64_t)t * tile, a1 = a0 + tile < n ? a0 + tile : n;
    float px[kTileUnroll], py[kTileUnroll], pz[kTileUnroll];
    bool on[kTileUnroll];
    auto load = [&](int64_t base) {
#pragma unroll
        for (int r = 0; r < kTileUnroll; ++r) {
            const int64_t i = base + threadIdx.x + r * kTileBlock;
            on[r] = i < a1;
            if (on[r]) {
                on[r] = alive[i] != 0;
                px[r] = rows[i];
                py[r] = rows[ld + i];
                pz[r] = rows[2 * ld + i];
            }
        }
    };
    /* the first round's loads do not depend on the box: in flight during
     * its reduction */
    load(a0);
    reduce_box(partial, n_partial, red, box_lds);
    if (blockIdx.x == 0 && threadIdx.x < 6) box[threadIdx.x] = box_lds[threadIdx.x];
    const Wrap w = plan_wrap(box_lds, k);
    for (int32_t p = threadIdx.x; p < parts; p += kTileBlock) cnt[p] = 0;
    __syncthreads();
    for (int64_t base = a0; base < a1; base += kTileAgents) {
        if (base != a0) load(base);
#pragma unroll
        for (int r = 0; r < kTileUnroll; ++r) {
            if (!on[r]) continue;
            uint32_t wx, wy, wz;
            wrapped_cell(w, px[r], py[r], pz[r], inv_h, wx, wy, wz);
            const uint32_t b = bucket_of(w, wx + 1, wy, wz);
            atomicAdd(&cnt[b >> s], 1);
            const int32_t g = ghost_offset(w, wx);
            if (g != 0) atomicAdd(&cnt[(uint32_t)((int32_t)b + g) >> s], 1);
        }
    }
    __syncthreads();
    for (int32_t p = threadIdx.x; p < parts; p += kTileBlock) hist[(int64_t)p * gridDim.x + t] = cnt[p];
}

__global__ void __launch_bounds__(kTileBlock) k_coll_part(const float* rows, int64_t ld, int64_t n,
                                                          const uint8_t* alive, const uint8_t* type, int n_types,
                                                          const float* radius, float inv_h, const int32_t* box,
                                                          int k, int s, int32_t parts, int64_t tile,
                                                          const int32_t* off, const int32_t* totals, float4* tpos,
                                                          int32_t* tid) {
    extern __shared__ int32_t cur[];
    const uint32_t t = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t a0 = (int64_t)t * tile, a1 = a0 + tile < n ? a0 + tile : n;
    /* all loads of a round first: the stores of the round may alias them as
     * far as the compiler knows; the first round's are in flight while the
     * cursors are read */
    float4 q[kTileUnroll];
    bool on[kTileUnroll];
    auto load = [&](int64_t base) {
#pragma unroll
        for (int r = 0; r < kTileUnroll; ++r) {
            const int64_t i = base + threadIdx.x + r * kTileBlock;
            on[r] = i < a1;
            if (on[r]) {
                on[r] = alive[i] != 0;
                q[r] = make_float4(rows[i], rows[ld + i], rows[2 * ld + i],
                                   radius[type ? type_entry(type, (uint32_t)i, n_types) : 0]);
            }
        }
    };
    load(a0);
    const Wrap w = plan_wrap(box, k);
    for (int32_t p = threadIdx.x; p < parts; p += kTileBlock) {
        const int64_t c = (int64_t)p * gridDim.x + t;
        cur[p] = off[c] + totals[c / kScanBlock];
    }
    __syncthreads();
    for (int64_t base = a0; base < a1; base += kTileAgents) {
        if (base != a0) load(base);
#pragma unroll
        for (int r = 0; r < kTileUnroll; ++r) {
            if (!on[r]) continue;
            const int32_t i = (int32_t)(base + threadIdx.x + r * kTileBlock);
            uint32_t wx, wy, wz;
            wrapped_cell(w, q[r].x, q[r].y, q[r].z, inv_h, wx, wy, wz);
            const uint32_t b = bucket_of(w, wx + 1, wy, wz);
            const int32_t slot = atomicAdd(&cur[b >> s], 1);
            tpos[slot] = q[r];
            tid[slot] = i;
            const int32_t g = ghost_offset(w, wx);
            if (g != 0) {
                const int32_t gslot = atomicAdd(&cur[(uint32_t)((int32_t)b + g) >> s], 1);
                tpos[gslot] = q[r];
                tid[gslot] = (int32_t)((uint32_t)i | 0x80000000u);
            }
        }
    }
}

/* Block b sorts window b (buckets [b kWindow, (b+1) kWindow)) of partition
 * b >> (s - kWindowBits), whose items sit in [off[p tiles], off[(p+1) tiles]).
 * A partition of at most kSortStage items is read once (each thread keeps
 * its items' buckets); the window's order is assembled in LDS as indices
 * into the partition, and the items are then copied out in that order, from
 * the L2, with consecutive stores.  A larger partition (a dense cluster, or
 * one of several windows) is read twice, to count and to place, and placed
 * by scattered stores. */
constexpr int kSortBlock = 512;
constexpr int kSortItems = 8;
constexpr int kSortStage = kSortBlock * kSortItems;
static_assert(kWindow % kSortBlock == 0, "whole rounds of the scan");
static_assert(kSortStage <= 65536, "staged indices are 16-bit");

__global__ void __launch_bounds__(kSortBlock) k_coll_sort(const float4* tpos, const int32_t* tid,
                                                          const int32_t* off, const int32_t* totals, int64_t tiles,
                                                          int64_t cells, float inv_h, const int32_t* box, int k,
                                                          int s, int32_t* start, float4* spos, int32_t* ids) {
    __shared__ int32_t cnt[kWindow];
    __shared__ uint16_t order[kSortStage];
    __shared__ int32_t wsum[kSortBlock / 64];
    const Wrap w = plan_wrap(box, k);
    const int64_t b0 = (int64_t)blockIdx.x << kWindowBits;
    const int64_t p = (int64_t)blockIdx.x >> (s - kWindowBits);
    const int32_t lo = cell_offset(off, totals, p * tiles, cells);
    const int32_t hi = cell_offset(off, totals, (p + 1) * tiles, cells);
    const bool staged = hi - lo <= kSortStage;      /* block-uniform */
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = threadIdx.x; j < kWindow; j += kSortBlock) cnt[j] = 0;
    __syncthreads();
    /* staged: bucket - b0 of item lo + threadIdx.x + u kSortBlock, or
     * kWindow when it is not in the window */
    int32_t rr[kSortItems];
    int32_t below = 0;
    if (staged) {
#pragma unroll
        for (int u = 0; u < kSortItems; ++u) {
            const int32_t j = lo + (int32_t)threadIdx.x + u * kSortBlock;
            rr[u] = kWindow;
            if (j >= hi) continue;
            const int64_t r = (int64_t)item_bucket(w, tpos[j], tid[j], inv_h) - b0;
            if (r < 0)
                ++below;
            else if (r < kWindow) {
                rr[u] = (int32_t)r;
                atomicAdd(&cnt[r], 1);
            }
        }
    } else {
        for (int32_t j = lo + (int32_t)threadIdx.x; j < hi; j += kSortBlock) {
            const int64_t r = (int64_t)item_bucket(w, tpos[j], tid[j], inv_h) - b0;
            if (r < 0)
                ++below;
            else if (r < kWindow)
                atomicAdd(&cnt[r], 1);
        }
    }
    for (int d = 32; d > 0; d >>= 1) below += __shfl_xor(below, d);
    if (lane == 0) wsum[wave] = below;
    __syncthreads();
    int32_t carry = lo;
    for (int u = 0; u < kSortBlock / 64; ++u) carry += wsum[u];
    const int32_t first = carry;                    /* the window's first slot */
    __syncthreads();
    /* exclusive scan of the window's counts, kSortBlock at a time: the
     * bucket starts, and the cursors of the placement below */
    for (int c = 0; c < kWindow; c += kSortBlock) {
        const int32_t v = cnt[c + threadIdx.x];
        int32_t x = v;
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t y = __shfl_up(x, d);
            if (lane >= d) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        int32_t pre = carry, all = 0;
        for (int u = 0; u < kSortBlock / 64; ++u) {
            pre += u < wave ? wsum[u] : 0;
            all += wsum[u];
        }
        const int32_t e = pre + x - v;
        cnt[c + threadIdx.x] = e;
        start[b0 + c + threadIdx.x] = e;
        carry += all;
        __syncthreads();
    }
    if (staged) {
        /* the window holds carry - first <= hi - lo <= kSortStage items */
#pragma unroll
        for (int u = 0; u < kSortItems; ++u) {
            if (rr[u] == kWindow) continue;
            order[atomicAdd(&cnt[rr[u]], 1) - first] = (uint16_t)(threadIdx.x + u * kSortBlock);
        }
        __syncthreads();
        for (int32_t j = threadIdx.x; j < carry - first; j += kSortBlock) {
            const int32_t from = lo + order[j];
            spos[first + j] = tpos[from];
            ids[first + j] = tid[from];
        }
    } else {
        for (int32_t j = lo + (int32_t)threadIdx.x; j < hi; j += kSortBlock) {
            const float4 qj = tpos[j];
            const int32_t ij = tid[j];
            const int64_t r = (int64_t)item_bucket(w, qj, ij, inv_h) - b0;
            if (r >= 0 && r < kWindow) {
                const int32_t slot = atomicAdd(&cnt[r], 1);
                spos[slot] = qj;
                ids[slot] = ij;
            }
        }
    }
}

/* One thread per sorted real slot (grid-stride; ghost slots are skipped):
 * consecutive lanes hold agents of the same or nearby cells, so the bucket
 * ranges and candidates they read are shared through the caches, and each
 * XCD takes a contiguous range of slots (xcd_tile).  The 9
 * candidate ranges are walked as one sequence, POTATO_QUERY_BATCH loads at
 * a time (indices past a lane's end read its own slot and are masked), and
 * a lane stops once it has found a collision.  (Copying each block's
 * candidate rows to LDS first, with consecutive loads, measured 1.25 times
 * slower at 1M agents: fewer waves per SIMD, a barrier per round, and the
 * L1 already serves most candidate reads.) */
__global__ void __launch_bounds__(256) k_coll_query(const float4* spos, const int32_t* ids, const int32_t* start,
                                                    const int32_t* total, float inv_h, const int32_t* box, int k_bits,
                                                    uint8_t* alive, int32_t* died_part) {
#pragma clang fp contract(off)
    __shared__ int32_t wave_died[256 / 64];
    int32_t my_died = 0;
    const Wrap w = plan_wrap(box, k_bits);
    const int64_t slots = *total;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    for (int64_t k0 = tile * blockDim.x; k0 < slots; k0 += stride) {
        /* whole blocks stay in the loop together, so the reduction below
         * sees every lane; slot indices stay below 2^31 (at most two slots
         * per agent, fewer than 2^30 agents) */
        const int32_t k = (int32_t)(k0 + threadIdx.x);
        const int32_t id = k < slots ? ids[k] : -1;
        bool hit = false;
        if (id >= 0) {
            const float4 pk = spos[k];
            uint32_t wx, wy, wz;
            wrapped_cell(w, pk.x, pk.y, pk.z, inv_h, wx, wy, wz);
            /* the 9 (y, z) rows: bucket range of columns wx .. wx + 2 (ghost-padded) */
            int32_t lo[9], hi[9];
#pragma unroll
            for (int r = 0; r < 9; ++r) {
                const uint32_t ry = (wy + (uint32_t)(r % 3) - 1u) & w.my;
                const uint32_t rz = (wz + (uint32_t)(r / 3) - 1u) & w.mz;
                const uint32_t b0 = bucket_of(w, wx, ry, rz);
                lo[r] = start[b0];
                hi[r] = start[b0 + 3];
            }
            /* candidate t of the sequence is slot t + d[r] for the last range r
             * whose first candidate number cum[r] is <= t */
            int32_t cum[9], d[9];
            int32_t T = 0;
#pragma unroll
            for (int r = 0; r < 9; ++r) {
                cum[r] = T;
                d[r] = lo[r] - T;
                T += hi[r] - lo[r];
            }
            auto collides = [&](const float4& pj) {
                const float ex = pk.x - pj.x, ey = pk.y - pj.y, ez = pk.z - pj.z;
                const float d2 = (ex * ex + ey * ey) + ez * ez;
                const float rs = pk.w + pj.w;
                return d2 < rs * rs;
            };
            constexpr int B = POTATO_QUERY_BATCH;
            for (int32_t t0 = 0; t0 < T && !hit; t0 += B) {
                float4 pc[B];
                bool use[B];
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    const int32_t t = t0 + u;
                    int32_t j = t + d[0];
#pragma unroll
                    for (int r = 1; r < 9; ++r) j = t >= cum[r] ? t + d[r] : j;
                    use[u] = t < T && j != k;
                    pc[u] = spos[t < T ? j : k];
                }
#pragma unroll
                for (int u = 0; u < B; ++u) hit |= use[u] && collides(pc[u]);
            }
            /* the query reads positions from the sorted copy only, so the
             * mask is updated in place */
            if (hit) alive[id] = 0;
        }
        my_died += hit ? 1 : 0;
    }
    /* agents marked dead by this block: a partial sum per block, added up by
     * k_coll_died (atomics on one counter serialise across the chip: one per
     * wave took most of the query's 0.21 ms at 1M agents; the last block
     * adding them up after a device-scope fence made the query 3.6 times
     * slower, one L2 write-back per block) */
    if (died_part) {
        int32_t x = my_died;
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
        if ((threadIdx.x & 63) == 0) wave_died[threadIdx.x / 64] = x;
        __syncthreads();
        if (threadIdx.x == 0) {
            int32_t sum = 0;
            for (int u = 0; u < (int)(blockDim.x / 64); ++u) sum += wave_died[u];
            died_part[blockIdx.x] = sum;
        }
    }
}

/* *died += the sum of the per-block counts of the query. */
__global__ void __launch_bounds__(256) k_coll_died(const int32_t* died_part, int n_part, unsigned long long* died) {
    __shared__ unsigned long long red[256 / 64];
    unsigned long long x = 0;
    for (int b = threadIdx.x; b < n_part; b += blockDim.x) x += (unsigned long long)died_part[b];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long sum = 0;
        for (int w = 0; w < (int)(blockDim.x / 64); ++w) sum += red[w];
        *died += sum;
    }
}

}  // namespace

namespace {

/* Bucket budget 2^k >= 2N, at least 2^10 (the wrap splits its k bits). */
constexpr int budget_bits(int64_t n) {
    int k = 10;
    while ((int64_t(1) << k) < 2 * n && k < 30) ++k;
    return k;
}

/* Buckets allocated: the budget plus the ghost columns (at most 2 per
 * 2^kMinXBits columns). */
constexpr int64_t buckets_alloc(int64_t n) {
    const int k = budget_bits(n);
    return (int64_t(1) << k) + (int64_t(1) << (k + 1 - kMinXBits));
}

/* Sizes of the two-level sort at N agents. */
struct SortPlan {
    int k;            /* bucket budget bits */
    int s;            /* log2 of the buckets per partition */
    int64_t parts;    /* partitions: parts << s >= m + 1, m the buckets allocated */
    int64_t tile;     /* agents per tile, a multiple of kTileAgents */
    int64_t tiles;    /* at most kMaxTiles */
};

constexpr SortPlan sort_plan(int64_t n) {
    SortPlan q{};
    q.k = budget_bits(n);
    const int64_t m1 = buckets_alloc(n) + 1;
    q.s = kWindowBits;
    while (((m1 + (int64_t(1) << q.s) - 1) >> q.s) > kMaxParts) ++q.s;
    q.parts = (m1 + (int64_t(1) << q.s) - 1) >> q.s;
    const int64_t per = (n + kTileAgents * kMaxTiles - 1) / (kTileAgents * kMaxTiles);
    q.tile = kTileAgents * (per < 1 ? 1 : per);
    q.tiles = (n + q.tile - 1) / q.tile;
    return q;
}

constexpr int64_t workspace_for(int64_t n) {
    const SortPlan q = sort_plan(n);
    const int64_t cells = q.parts * q.tiles;
    const int64_t chunks = (cells + kScanBlock - 1) / kScanBlock;
    /* items (x, y, z, r) in partition order and in bucket order [2n] each
     * first (16-byte aligned: agents and ghosts); their ids [2n] each;
     * bucket starts [parts << s]; partition-tile offsets [parts * tiles + 1];
     * chunk totals of their scan [chunks]; bounding box [6]; its per-block
     * partials [kBoxBlocks][6]; the query's per-block counts of dead agents */
    const int64_t blocks = (n + 255) / 256;
    return 16 * 4 * n + 4 * (4 * n + (q.parts << q.s) + cells + 1 + chunks + 6 + 6 * kBoxBlocks + blocks) + 256;
}

/* Workspace of the allocation-free entry point: a file-scope device array
 * sized for the largest swarm it accepts.  Every GPU the library runs on
 * holds its own copy until the process ends; host code reaches it only
 * through the address hipGetSymbolAddress returns for the current device
 * (the array's name in host code is not a device address). */
constexpr int64_t kNoAllocBytes = workspace_for(kNoAllocMaxAgents);

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

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
    const SortPlan q = sort_plan(n);
    const int64_t cells = q.parts * q.tiles;
    float4* tpos = reinterpret_cast<float4*>(workspace);
    float4* spos = tpos + 2 * n;
    int32_t* tid = reinterpret_cast<int32_t*>(spos + 2 * n);
    int32_t* ids = tid + 2 * n;
    int32_t* start = ids + 2 * n;
    int32_t* off = start + (q.parts << q.s);
    int32_t* totals = off + cells + 1;
    int32_t* box = totals + scan_chunks((uint32_t)cells);
    int32_t* partial = box + 6;
    int32_t* died_part = partial + 6 * kBoxBlocks;
    const float inv_h = 1.0f / (2.02f * r_max);
    const unsigned nb = (unsigned)((n + 255) / 256);
    const unsigned nbox = nb < (unsigned)kBoxBlocks ? nb : (unsigned)kBoxBlocks;
    const size_t lds = (size_t)q.parts * sizeof(int32_t);
    hipLaunchKernelGGL(k_coll_bounds, dim3(nbox), dim3(256), 0, s, rows, ld, n, alive, inv_h, partial);
    hipLaunchKernelGGL(k_coll_hist, dim3((unsigned)q.tiles), dim3(kTileBlock), lds, s, rows, ld, n, alive, inv_h,
                       partial, (int)nbox, box, q.k, q.s, (int32_t)q.parts, q.tile, off);
    /* in place, chunk by chunk (the consumers add the chunk totals); the
     * slot count goes to off[cells] */
    launch_exclusive_scan_chunks(off, off, totals, off + cells, (uint32_t)cells, s);
    hipLaunchKernelGGL(k_coll_part, dim3((unsigned)q.tiles), dim3(kTileBlock), lds, s, rows, ld, n, alive, type,
                       n_types, radius_dev, inv_h, box, q.k, q.s, (int32_t)q.parts, q.tile, off, totals, tpos, tid);
    hipLaunchKernelGGL(k_coll_sort, dim3((unsigned)((q.parts << q.s) >> kWindowBits)), dim3(kSortBlock), 0, s, tpos,
                       tid, off, totals, q.tiles, cells, inv_h, box, q.k, q.s, start, spos, ids);
    hipLaunchKernelGGL(k_coll_query, dim3(nb), dim3(256), 0, s, spos, ids, start, off + cells, inv_h, box, q.k, alive,
                       died ? died_part : nullptr);
    if (died) hipLaunchKernelGGL(k_coll_died, dim3(1), dim3(256), 0, s, died_part, (int)nb, died);
    return hipGetLastError();
}

}  // namespace potato
