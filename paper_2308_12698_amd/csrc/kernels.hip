/*
 * kernels.hip -- gfx950 kernels of the batched quadrotor step.
 *
 * k_rollout: one agent per lane, its 30-float state (and, with CARRY, its
 * 10 rounding carries) loaded once into registers (coalesced
 * structure-of-arrays rows), advanced n_steps time steps, stored once.  With n_steps = 1 and one agent per thread this is
 * the plain per-step form (HBM bound: the state round-trips every step);
 * with many steps per launch it is the fused form (VALU bound).  A
 * grid-stride loop lets a launch use a persistent grid.  Optional pieces
 * are template switches so that the homogeneous path carries no per-agent
 * type or gain traffic:
 *   HET   per-agent type index into the type table staged in LDS (the
 *         paper runs one process per type, Sec. II-A; here all types share
 *         one launch);
 *   GAINS per-agent controller gains;
 *   CKPT  checkpoints every ckpt_every steps for the adjoint (always with
 *         CARRY: the adjoint replays the compensated integrator);
 *   PERM  processing order (agents grouped by type); without it, a
 *         launch whose types fall into 2-8 classes of equal budget and
 *         kind sorts each block's agents by class in LDS and hands the
 *         64-agent groups to its waves (group_agents);
 *   CARRY rounding carries of p, v, J and the position-loop integral kept
 *         in the caller's carry rows (without: uncompensated updates);
 *   KINDS the type table also holds cars and fixed-wing aircraft: a lane
 *         whose type is one of those runs its own step (vehicle_step.h)
 *         over rows 0-6 instead of the quadrotor's.
 * k_adjoint: reverse sweep of a checkpointed rollout, one agent per lane,
 * each segment recomputed into a per-wave tape and then reversed;
 * k_adjoint_pipe: the same sweep for small swarms, a recomputing and a
 * reversing wave per 64 agents.  k_block_hist / k_scatter: the processing
 * order by type.  k_count_nonfinite: agents with a NaN or infinite row.
 * No MFMA: nothing in a quadrotor step is a dense contraction.
 */
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "kernels.h"
#include "quad_adjoint.h"
#include "scan.h"
#include "vehicle_step.h"

namespace potato {

namespace {

/* Where the step reads the launch's limits and time-step constants from:
 * 0 (default) keeps them as kernel arguments in scalar registers; 2 reads
 * the three that the RK4 stages use ~50 times per step (dt, dt/2, dt/6)
 * from the LDS copy into vector registers; 1 reads all of them from LDS
 * (the extra vector registers then spill at 4 waves per SIMD).  A VALU
 * instruction with a scalar-register operand issues at half the rate of one
 * with vector operands only on gfx950 (measured: 62 against 93-107 lanes
 * per clock per CU), but the step is latency bound at its occupancy: 2
 * removes 53 such operands per step and measured no faster. */
#ifndef POTATO_LIMITS_FROM_LDS
#define POTATO_LIMITS_FROM_LDS 0
#endif
/* Occupancy target of the rollout kernel in waves per SIMD (0 = compiler's
 * choice).  More resident waves hide the latency of dependent FP32 chains
 * and transcendental ops; the closed-loop kernel fits 4 waves (121-127
 * VGPRs) without spilling, 5 waves spill. */
#ifndef POTATO_ROLLOUT_WAVES
#define POTATO_ROLLOUT_WAVES 4
#endif
#if POTATO_ROLLOUT_WAVES > 0
#define POTATO_ROLLOUT_ATTR __attribute__((amdgpu_waves_per_eu(POTATO_ROLLOUT_WAVES, POTATO_ROLLOUT_WAVES)))
#else
#define POTATO_ROLLOUT_ATTR
#endif

/* The per-type constants (and the launch's limits) are staged in LDS and
 * read from there by every lane, also when all agents share one type:
 * values loaded from LDS live in vector registers, and the step's FMAs then
 * take them as vector operands.  As scalar-register operands of the same
 * instructions (kernel arguments) the step measured 16-20 % slower. */
__device__ __forceinline__ void stage_constants(const TypeConst* table, int n_types, const Limits& lim,
                                                TypeConst* tab, Limits* l) {
    const int words = n_types * (int)(sizeof(TypeConst) / 4);
    const uint32_t* src = reinterpret_cast<const uint32_t*>(table);
    uint32_t* dst = reinterpret_cast<uint32_t*>(tab);
    for (int i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
    if (threadIdx.x == 0) *l = lim;
    __syncthreads();
}

/* Advance one car or fixed-wing agent (byte offset bo into the rows)
 * `steps` time steps from rows 0-6 and their carries (carry row k holds the
 * carry of state row k), store them, and return its final position in p. */
template <int KIND, int MODE, bool CARRY>
__device__ __forceinline__ void advance_vehicle(const StepArgs& A, const VehConst& c, const Limits& lim,
                                                uint32_t bo, int steps, float p[3]) {
    float* const R = A.rows;
    const int64_t ld = A.ld;
    auto row = [&](int k) -> float& { return elem(uniform(R + k * ld), bo); };
    auto crow = [&](int k) -> float& { return elem(uniform(A.carry + k * A.carry_ld), bo); };
    float x[7], lo[7], u[3] = {0.0f, 0.0f, 0.0f}, wp[3];
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        x[k] = veh_row<KIND>(k) ? row(k) : 0.0f;
        lo[k] = CARRY && veh_row<KIND>(k) ? crow(k) : 0.0f;
    }
    int64_t next_epoch_step = INT64_MAX;
    int epoch = 0;
    if (MODE == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) u[k] = elem(uniform(A.motor_cmd + k * A.cmd_ld), bo);
    } else {
        if (A.resample > 0) {
            const int64_t e0 = A.step0 / A.resample;
            epoch = e0 < A.n_epochs - 1 ? (int)e0 : A.n_epochs - 1;
            next_epoch_step = e0 < A.n_epochs - 1 ? (e0 + 1) * A.resample : INT64_MAX;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) wp[k] = elem(uniform(A.wp + ((int64_t)epoch * 3 + k) * A.cmd_ld), bo);
    }
    for (int s = 0; s < steps; ++s) {
        if (MODE == 1) {
            if (A.step0 + s == next_epoch_step) {
                ++epoch;
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    wp[k] = elem(uniform(A.wp + ((int64_t)epoch * 3 + k) * A.cmd_ld), bo);
                next_epoch_step = epoch < A.n_epochs - 1 ? next_epoch_step + A.resample : INT64_MAX;
            }
        }
        VehTrig T;
        veh_trig<KIND>(x, T);
        if (MODE == 1) veh_guidance<KIND>(c, x, T, wp, u);
        veh_rk4<KIND, CARRY>(c, lim, x, T, lo, u);
    }
#pragma unroll
    for (int k = 0; k < 7; ++k)
        if (veh_row<KIND>(k)) row(k) = x[k];
    if (CARRY) {
#pragma unroll
        for (int k = 0; k < 7; ++k)
            if (veh_row<KIND>(k)) crow(k) = lo[k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) p[k] = x[k];
}

/* Grouping a block's agents by class (a launch with a per-agent type and
 * no processing order, whose types fall into 2..kMaxGroups classes of equal
 * step budget and kind).  The block sorts a chunk of up to kGroupWidths
 * block widths of consecutive agents by class, stably, from wave ballots
 * and a prefix over the (width, wave) cells' counts.  Each class's agents
 * fill whole groups of 64 first; what is left of each class (fewer than 64)
 * is packed with the leftovers of the other classes of its kind, longest
 * budget first, so that a group never holds two kinds (the gaps hold -1)
 * and a rare class does not cost a whole group of its own.  Classes are
 * numbered longest step first, and the groups are handed out in the order
 * of the class of their first agent, so that the groups handed out last are
 * short. */
struct GroupLds {
    int32_t* count;   /* [cells][kMaxGroups] agents of each class per (width, wave) cell */
    int32_t* first;   /* [cells][kMaxGroups] rank in its class of the cell's first agent */
    int32_t* slot;    /* [kGroupWidths * B + kMaxGroups * 64] offset from base, or -1 */
    int32_t* order;   /* [kGroupWidths * B / 64 + kMaxGroups] groups in hand-out order */
    int32_t* head;    /* [kGroupWidths * B / 64 + kMaxGroups] class of each group's first agent */
    int32_t* cls;     /* [kMaxGroups][4] class total, kind, start of its whole groups, of its leftover */
    int32_t* misc;    /* [0] groups of 64 that hold an agent, [1] the next one to hand out */
};

__device__ __forceinline__ GroupLds group_lds(int32_t* area, int B) {
    const int cells = kGroupWidths * (B / 64) * kMaxGroups;
    const int groups = kGroupWidths * (B / 64) + kMaxGroups;
    GroupLds L;
    L.count = area;
    L.first = area + cells;
    L.slot = area + 2 * cells;
    L.order = L.slot + kGroupWidths * B + kMaxGroups * 64;
    L.head = L.order + groups;
    L.cls = L.head + groups;
    L.misc = L.cls + 4 * kMaxGroups;
    return L;
}

/* Sort the chunk [base, end) (ch block widths, ch <= kGroupWidths).
 * Afterwards slot[p] is the offset from base of the agent at sorted
 * position p, order[] the groups of 64 in hand-out order, misc[0] their
 * number and misc[1] = 0.  Contains barriers: every thread of the block
 * calls it with the same arguments. */
__device__ __forceinline__ void group_agents(const StepArgs& A, const TypeConst* tab, int64_t base, int64_t end,
                                             int ch, const GroupLds& L) {
    const int B = blockDim.x, t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63, n_waves = B >> 6, n_cells = ch * n_waves, nk = A.n_groups;
    const uint64_t below = (uint64_t(1) << lane) - 1;
    int key[kGroupWidths];
    uint64_t same[kGroupWidths];
#pragma unroll
    for (int c = 0; c < kGroupWidths; ++c) {
        key[c] = kMaxGroups;                      /* past the end: not placed */
        same[c] = 0;
        if (c < ch) {
            const int64_t j = base + (int64_t)c * B + t;
            if (j < end) key[c] = tab[type_entry(A.type, (uint32_t)j, A.n_types)].group;
            int32_t* cnt = L.count + (c * n_waves + wave) * kMaxGroups;
#pragma unroll
            for (int k = 0; k < kMaxGroups; ++k) {
                if (k < nk) {
                    const uint64_t m = __ballot(key[c] == k);
                    if (key[c] == k) same[c] = m;
                    if (lane == 0) cnt[k] = __popcll(m);
                }
            }
        }
    }
    __syncthreads();
    /* every wave has left the previous chunk's hand-out loop.  Class t: its
     * cells' ranks within the class, its total and its kind */
    if (t < nk) {
        int32_t run = 0;
        for (int cell = 0; cell < n_cells; ++cell) {
            L.first[cell * kMaxGroups + t] = run;
            run += L.count[cell * kMaxGroups + t];
        }
        int kind = 0;
        for (int ty = 0; ty < A.n_types; ++ty)
            if (tab[ty].group == t) kind = tab[ty].kind;
        L.cls[4 * t + 0] = run;
        L.cls[4 * t + 1] = kind;
    }
    if (t == 0) L.misc[1] = 0;
    for (int p = t; p < ch * B + nk * 64; p += B) L.slot[p] = -1;
    __syncthreads();
    if (t == 0) {
        /* whole groups class by class, then the leftovers kind by kind
         * (kinds in the order of their longest class), each kind's run
         * rounded up to 64 */
        int32_t pos = 0;
        for (int k = 0; k < nk; ++k) {
            L.cls[4 * k + 2] = pos;
            pos += L.cls[4 * k] & ~63;
        }
        uint32_t placed = 0;
        for (int k0 = 0; k0 < nk; ++k0) {
            if (placed >> k0 & 1u) continue;
            const int kind = L.cls[4 * k0 + 1];
            for (int k = k0; k < nk; ++k) {
                if (L.cls[4 * k + 1] != kind) continue;
                placed |= 1u << k;
                L.cls[4 * k + 3] = pos;
                pos += L.cls[4 * k] & 63;
            }
            pos = (pos + 63) & ~63;
        }
        L.misc[0] = pos >> 6;
    }
    __syncthreads();
    const int n_out = L.misc[0];
    /* each group's first agent's class (a group never starts in a gap) */
    for (int g = t; g < n_out; g += B) {
        const int32_t p0 = g * 64;
        int h = 0;
        for (int k = 0; k < nk; ++k) {
            const int32_t total = L.cls[4 * k], whole = L.cls[4 * k + 2], left = L.cls[4 * k + 3];
            if ((p0 >= whole && p0 < whole + (total & ~63)) || (p0 >= left && p0 < left + (total & 63))) h = k;
        }
        L.head[g] = h;
    }
#pragma unroll
    for (int c = 0; c < kGroupWidths; ++c)
        if (c < ch && key[c] < nk) {
            const int k = key[c];
            const int32_t q = L.first[(c * n_waves + wave) * kMaxGroups + k] + __popcll(same[c] & below);
            const int32_t whole = L.cls[4 * k] & ~63;
            L.slot[q < whole ? L.cls[4 * k + 2] + q : L.cls[4 * k + 3] + (q - whole)] = c * B + t;
        }
    __syncthreads();
    /* hand-out order: by the class of the first agent, then by position */
    for (int g = t; g < n_out; g += B) {
        const int h = L.head[g];
        int r = 0;
        for (int u = 0; u < n_out; ++u) {
            const int hu = L.head[u];
            r += (hu < h || (hu == h && u < g)) ? 1 : 0;
        }
        L.order[r] = g;
    }
    __syncthreads();
    /* the next call writes these arrays only after a barrier that every
     * thread reaches once it is done with this call's */
}

template <int MODE, bool HET, bool GAINS, bool CKPT, bool PERM, bool CARRY, bool KINDS>
__global__ void __launch_bounds__(1024) POTATO_ROLLOUT_ATTR k_rollout(const StepArgs A) {
    static_assert(!(KINDS && CKPT), "checkpoints (the adjoint) cover quadrotors only");
    static_assert(CARRY || !CKPT, "checkpoints hold the carries");
    extern __shared__ float4 lds_raw[];
    Limits* lim_lds = reinterpret_cast<Limits*>(lds_raw);
    TypeConst* tab = reinterpret_cast<TypeConst*>(lds_raw + (sizeof(Limits) + 15) / 16);
    stage_constants(A.table, A.n_types, A.lim, tab, lim_lds);
#if POTATO_LIMITS_FROM_LDS == 1
    const Limits& lim = *lim_lds;
#elif POTATO_LIMITS_FROM_LDS == 2
    Limits lim = A.lim;
    lim.dt = lim_lds->dt; lim.half_dt = lim_lds->half_dt; lim.dt6 = lim_lds->dt6;
#else
    const Limits& lim = A.lim;
#endif
    const int64_t ld = A.ld;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    /* One agent's whole launch. */
    auto advance = [&](int64_t j) {
        /* agent index < 2^30, so byte offsets into rows fit 32 bits.  Row
         * addresses are uniform: every active lane starts at step 0 and
         * steps together, so the epoch and checkpoint slot agree too. */
        const uint32_t i = PERM ? order_entry(A.perm, (uint32_t)j, A.n) : (uint32_t)j;
        const uint32_t bo = i << 2;
        const TypeConst& c = HET ? tab[type_entry(A.type, i, A.n_types)] : tab[0];
        float* const R = A.rows;
        auto row = [&](int k) -> float& { return elem(uniform(R + k * ld), bo); };
        auto crow = [&](int k) -> float& { return elem(uniform(A.carry + k * A.carry_ld), bo); };
        /* position snapshot (rows 0-2, [3][n]) written straight to mapped host
         * memory; never requested together with checkpoints, and left out of
         * those variants (whose step loop has no scalar registers to spare) */
        const bool snapshot = !CKPT && A.snap != nullptr;
        auto snap = [&](int k) -> float& { return elem(uniform(A.snap + k * A.n), bo); };
        /* an agent that is not advanced keeps its stored position */
        auto snap_stored = [&]() {
            if (snapshot) {
#pragma unroll
                for (int k = 0; k < 3; ++k) snap(k) = row(k);
            }
        };
        if (A.alive && !elem(A.alive, i)) {
            snap_stored();
            return;
        }

        int64_t left = (int64_t)c.budget - A.step0;
        left = left < 0 ? 0 : left;
        const int steps = left < A.n_steps ? (int)left : A.n_steps;
        if (steps == 0) {
            snap_stored();
            return;
        }
        if (KINDS && c.kind != KIND_QUAD) {
            float pf[3];
            if (c.kind == KIND_CAR)
                advance_vehicle<KIND_CAR, MODE, CARRY>(A, c.veh, lim, bo, steps, pf);
            else
                advance_vehicle<KIND_WING, MODE, CARRY>(A, c.veh, lim, bo, steps, pf);
            if (snapshot) {
#pragma unroll
                for (int k = 0; k < 3; ++k) snap(k) = pf[k];
            }
            return;
        }

        Agent a;
#pragma unroll
        for (int k = 0; k < 3; ++k) { a.p[k] = row(k); a.v[k] = row(3 + k); a.w[k] = row(10 + k); }
#pragma unroll
        for (int k = 0; k < 4; ++k) { a.q[k] = row(6 + k); a.d[k] = row(13 + k); }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            a.p_lo[k] = CARRY ? crow(k) : 0.0f;
            a.v_lo[k] = CARRY ? crow(3 + k) : 0.0f;
        }
        if (MODE == 1) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                a.ip[k] = row(17 + k); a.ia[k] = row(20 + k);
                a.ir[k] = row(23 + k); a.wprev[k] = row(26 + k);
            }
            a.J = row(29);
            a.J_lo = CARRY ? crow(6) : 0.0f;
#pragma unroll
            for (int k = 0; k < 3; ++k) a.ip_lo[k] = CARRY ? crow(7 + k) : 0.0f;
        } else {
#pragma unroll
            for (int k = 0; k < 3; ++k) { a.ip[k] = a.ia[k] = a.ir[k] = a.wprev[k] = a.ip_lo[k] = 0.0f; }
            a.J = a.J_lo = 0.0f;
        }

        Gains g;
        if (GAINS) {
            const float* G = A.gains;
            const int64_t gl = A.gains_ld;
            auto gain = [&](int k) { return elem(uniform(G + k * gl), bo); };
            g = Gains{gain(0), gain(1), gain(2), gain(3), gain(4), gain(5), gain(6), gain(7), gain(8)};
        } else {
            g = Gains{c.gains[0], c.gains[1], c.gains[2], c.gains[3], c.gains[4],
                      c.gains[5], c.gains[6], c.gains[7], c.gains[8]};
        }
        g.kdr_dt = g.kdr * lim.inv_dt;

        float dc[4];
        float wp[3];
        int64_t next_epoch_step = INT64_MAX;
        int epoch = 0;
        if (MODE == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) dc[k] = elem(uniform(A.motor_cmd + k * A.cmd_ld), bo);
        } else {
            if (A.resample > 0) {
                const int64_t e0 = A.step0 / A.resample;
                epoch = e0 < A.n_epochs - 1 ? (int)e0 : A.n_epochs - 1;
                next_epoch_step = e0 < A.n_epochs - 1 ? (e0 + 1) * A.resample : INT64_MAX;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) wp[k] = elem(uniform(A.wp + ((int64_t)epoch * 3 + k) * A.cmd_ld), bo);
        }
        int ck_next = 0, ck_slot = 0;
        if (CKPT) {
            ck_slot = (A.k0 + A.ckpt_every - 1) / A.ckpt_every;
            ck_next = ck_slot * A.ckpt_every - A.k0;
        }

        for (int s = 0; s < steps; ++s) {
            if (CKPT && s == ck_next) {
                float* const O = A.ckpt + (int64_t)ck_slot * kCkptRows * ld;
                auto out = [&](int k) -> float& { return elem(uniform(O + k * ld), bo); };
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    out(k) = a.p[k]; out(3 + k) = a.v[k]; out(10 + k) = a.w[k];
                    out(17 + k) = a.ip[k]; out(20 + k) = a.ia[k];
                    out(23 + k) = a.ir[k]; out(26 + k) = a.wprev[k];
                    out(30 + k) = a.p_lo[k]; out(33 + k) = a.v_lo[k];
                    out(37 + k) = a.ip_lo[k];
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) { out(6 + k) = a.q[k]; out(13 + k) = a.d[k]; }
                out(29) = a.J;
                out(36) = a.J_lo;
                ++ck_slot;
                ck_next += A.ckpt_every;
            }
            if (MODE == 1) {
                if (A.step0 + s == next_epoch_step) {
                    ++epoch;
#pragma unroll
                    for (int k = 0; k < 3; ++k)
                        wp[k] = elem(uniform(A.wp + ((int64_t)epoch * 3 + k) * A.cmd_ld), bo);
                    next_epoch_step = epoch < A.n_epochs - 1 ? next_epoch_step + A.resample : INT64_MAX;
                }
                controller<CARRY>(c, lim, g, a, wp, dc);
            }
            rk4_step<CARRY>(c, lim, a, dc);
        }

#pragma unroll
        for (int k = 0; k < 3; ++k) { row(k) = a.p[k]; row(3 + k) = a.v[k]; row(10 + k) = a.w[k]; }
#pragma unroll
        for (int k = 0; k < 4; ++k) { row(6 + k) = a.q[k]; row(13 + k) = a.d[k]; }
        if (CARRY) {
#pragma unroll
            for (int k = 0; k < 3; ++k) { crow(k) = a.p_lo[k]; crow(3 + k) = a.v_lo[k]; }
        }
        if (MODE == 1) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                row(17 + k) = a.ip[k]; row(20 + k) = a.ia[k];
                row(23 + k) = a.ir[k]; row(26 + k) = a.wprev[k];
            }
            row(29) = a.J;
            if (CARRY) {
                crow(6) = a.J_lo;
#pragma unroll
                for (int k = 0; k < 3; ++k) crow(7 + k) = a.ip_lo[k];
            }
        }
        if (snapshot) {
#pragma unroll
            for (int k = 0; k < 3; ++k) snap(k) = a.p[k];
        }
    };
    if constexpr (HET && !PERM && !CKPT) {
        /* a per-agent type in the caller's order: each block owns
         * ceil(n / grid) consecutive agents (a multiple of 64) and steps
         * them in groups of 64.  When the types fall into classes (equal
         * step budget and kind), the groups are sorted by class, chunk by
         * chunk of up to kGroupWidths block widths, so that a wave's 64
         * agents take the same number of steps of the same kind's loop
         * instead of waiting for the longest budget and running every
         * kind's loop in turn; the block's waves then take the groups in
         * turn, so that they finish together.  Otherwise wave w steps the
         * chunk's group w.  An agent's arithmetic does not depend on its
         * lane, so the results are the same bits either way.  The chunk
         * loop's bounds and `grouped` are the same for the whole block, so
         * every thread reaches the barriers. */
        const bool grouped = A.n_groups >= 2;
        const GroupLds L = group_lds(reinterpret_cast<int32_t*>(tab + A.n_types), blockDim.x);
        const int64_t B = blockDim.x;
        const int64_t width = grouped ? kGroupWidths * B : B;
        const int64_t per_block = ((A.n + gridDim.x - 1) / gridDim.x + 63) / 64 * 64;
        const int64_t lo = (int64_t)blockIdx.x * per_block;
        const int64_t hi = lo + per_block < A.n ? lo + per_block : A.n;
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, n_waves = blockDim.x >> 6;
        auto take = [&]() {
            int g = 0;
            if (lane == 0) g = atomicAdd(&L.misc[1], 1);
            return __builtin_amdgcn_readfirstlane(g);
        };
        for (int64_t base = lo; base < hi; base += width) {
            const int64_t end = base + width < hi ? base + width : hi;
            int n_out = (int)((end - base + 63) / 64);
            if (grouped) {
                group_agents(A, tab, base, end, (int)((end - base + B - 1) / B), L);
                n_out = L.misc[0];
            }
            for (int g = grouped ? take() : wave; g < n_out; g = grouped ? take() : g + n_waves) {
                const int32_t off = grouped ? L.slot[L.order[g] * 64 + lane] : g * 64 + lane;
                if (off >= 0 && base + off < end) advance(base + off);
            }
        }    } else {
        for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < A.n; j += stride) advance(j);
    }

}

/* Reverse sweep of the checkpointed closed-loop rollout: one agent per lane
 * (grid-stride), cotangents and gain sums in registers, the recomputed
 * segment in this wave's tape blocks.  Two waves per SIMD: the hot loops
 * fit 256 registers without spills (one wave leaves the tape loads exposed). */
#ifndef POTATO_ADJOINT_WAVES
#define POTATO_ADJOINT_WAVES 2
#endif
/* Limits of the adjoint: same choices as the rollout's POTATO_LIMITS_FROM_LDS. */
#ifndef POTATO_ADJOINT_LIMITS_FROM_LDS
#define POTATO_ADJOINT_LIMITS_FROM_LDS 0
#endif

template <bool HET, bool GAINS, bool PERM>
__global__ void __launch_bounds__(kAdjBlock)
    __attribute__((amdgpu_waves_per_eu(POTATO_ADJOINT_WAVES, POTATO_ADJOINT_WAVES))) k_adjoint(const AdjArgs A) {
    extern __shared__ float4 lds_raw[];
    Limits* lim_lds = reinterpret_cast<Limits*>(lds_raw);
    TypeConst* tab = reinterpret_cast<TypeConst*>(lds_raw + (sizeof(Limits) + 15) / 16);
    stage_constants(A.table, A.n_types, A.lim, tab, lim_lds);
#if POTATO_ADJOINT_LIMITS_FROM_LDS == 1
    const Limits& lim = *lim_lds;
#elif POTATO_ADJOINT_LIMITS_FROM_LDS == 2
    Limits lim = A.lim;
    lim.dt = lim_lds->dt; lim.half_dt = lim_lds->half_dt; lim.dt6 = lim_lds->dt6;
#else
    const Limits& lim = A.lim;
#endif
    const int64_t ld = A.ld;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    /* this wave's tape blocks: kTapeRows x 64 floats per step, waves side by side */
    const int64_t wave = tid >> 6;
    const uint32_t lb = (uint32_t)(tid & 63) << 2;
    float* const tape = A.tape + wave * (int64_t)kTapeRows * 64;
    const int64_t tape_step = (stride >> 6) * (int64_t)kTapeRows * 64;
    const int n_seg_all = (A.n_steps + A.K - 1) / A.K;
    for (int64_t j = tid; j < A.n; j += stride) {
        const uint32_t i = PERM ? order_entry(A.perm, (uint32_t)j, A.n) : (uint32_t)j;
        const uint32_t bo = i << 2;
        const TypeConst& c = HET ? tab[type_entry(A.type, i, A.n_types)] : tab[0];
        int64_t left = (int64_t)c.budget - A.step0;
        left = left < 0 ? 0 : left;
        int steps = left < A.n_steps ? (int)left : A.n_steps;
        if (A.alive && !elem(A.alive, i)) steps = 0;      /* dead: identity map */
        Gains g;
        if (GAINS) {
            const float* G = A.gains;
            const int64_t gl = A.gains_ld;
            auto gain = [&](int k) { return elem(G + k * gl, bo); };
            g = Gains{gain(0), gain(1), gain(2), gain(3), gain(4), gain(5), gain(6), gain(7), gain(8)};
        } else {
            g = Gains{c.gains[0], c.gains[1], c.gains[2], c.gains[3], c.gains[4],
                      c.gains[5], c.gains[6], c.gains[7], c.gains[8]};
        }
        g.kdr_dt = g.kdr * lim.inv_dt;
        AgentAdj lam;
        load_adj(A.grad_final, ld, bo, lam);
        float gk[9] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        if (steps > 0)
            agent_backward(c, lim, g, A.ckpt, ld, bo, A.K, n_seg_all, steps, A.step0, A.wp, A.cmd_ld,
                           A.n_epochs, A.resample, tape, tape_step, lb, lam, gk);
        store_adj(A.grad_x0, A.grad_mem, ld, bo, lam);
        if (A.grad_gains) {
#pragma unroll
            for (int k = 0; k < 9; ++k) elem(A.grad_gains + k * ld, bo) = gk[k];
        }
    }
}

/*
 * Pipelined reverse sweep for swarms too small to give every SIMD two
 * waves of the kernel above: a block of two waves serves 64 agents, wave 0
 * recomputing segment s - 1 into one tape buffer while wave 1 reverses
 * segment s from the other, one block barrier per segment.  Each wave
 * performs the same operations as the one-wave-per-agent kernel, so the
 * gradients are bitwise the same.  The segment loop and its barrier are
 * outside every per-lane condition, and every iteration of every agent
 * group reaches the barrier in both waves (ceil(n_steps / K) + 1 per
 * group, the group loop bounds being the same for the whole block).
 * Tape: per block, 2 buffers x K slots x kTapeRows x 64 floats.
 */
template <bool HET, bool GAINS, bool PERM>
__global__ void __launch_bounds__(kAdjPipeBlock)
    __attribute__((amdgpu_waves_per_eu(POTATO_ADJOINT_WAVES, POTATO_ADJOINT_WAVES))) k_adjoint_pipe(const AdjArgs A) {
    extern __shared__ float4 lds_raw[];
    Limits* lim_lds = reinterpret_cast<Limits*>(lds_raw);
    TypeConst* tab = reinterpret_cast<TypeConst*>(lds_raw + (sizeof(Limits) + 15) / 16);
    stage_constants(A.table, A.n_types, A.lim, tab, lim_lds);
    const Limits& lim = A.lim;
    const int64_t ld = A.ld;
    const bool producer = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) == 0;
    /* the reversing wave is the critical path (the recomputing wave waits
     * for it at every segment barrier): it issues first whenever both are
     * ready on a SIMD */
    if (!producer) __builtin_amdgcn_s_setprio(3);
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t lb = lane << 2;
    const int64_t tape_step = (int64_t)kTapeRows * 64;
    const int64_t buf_stride = (int64_t)A.K * tape_step;
    float* const tape = A.tape + (int64_t)blockIdx.x * 2 * buf_stride;
    const int n_seg_all = (A.n_steps + A.K - 1) / A.K;
    const int64_t n_groups = (A.n + 63) >> 6;
    for (int64_t grp = blockIdx.x; grp < n_groups; grp += gridDim.x) {
        const int64_t j = (grp << 6) + lane;
        const bool valid = j < A.n;
        const uint32_t i = !valid ? 0u : PERM ? order_entry(A.perm, (uint32_t)j, A.n) : (uint32_t)j;
        const uint32_t bo = i << 2;
        const TypeConst& c = HET ? tab[type_entry(A.type, i, A.n_types)] : tab[0];
        int64_t left = (int64_t)c.budget - A.step0;
        left = left < 0 ? 0 : left;
        int steps = left < A.n_steps ? (int)left : A.n_steps;
        if (!valid || (A.alive && !elem(A.alive, i))) steps = 0;
        const int n_seg = (steps + A.K - 1) / A.K;
        Gains g;
        if (GAINS) {
            const float* G = A.gains;
            const int64_t gl = A.gains_ld;
            auto gain = [&](int k) { return elem(G + k * gl, bo); };
            g = Gains{gain(0), gain(1), gain(2), gain(3), gain(4), gain(5), gain(6), gain(7), gain(8)};
        } else {
            g = Gains{c.gains[0], c.gains[1], c.gains[2], c.gains[3], c.gains[4],
                      c.gains[5], c.gains[6], c.gains[7], c.gains[8]};
        }
        g.kdr_dt = g.kdr * lim.inv_dt;
        WaypointCache wc{A.wp, A.cmd_ld, A.n_epochs, bo};
        AgentAdj lam;
        float gk[9] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        if (!producer && valid) load_adj(A.grad_final, ld, bo, lam);
        /* iteration t: wave 0 recomputes segment n_seg_all - 1 - t into
         * buffer (segment & 1), wave 1 reverses segment n_seg_all - t,
         * recomputed in the previous iteration, from the other buffer */
        for (int t = 0; t <= n_seg_all; ++t) {
            if (producer) {
                const int seg = n_seg_all - 1 - t;
                if (seg >= 0 && seg < n_seg)
                    recompute_segment(c, lim, g, A.ckpt, ld, bo, A.K, seg, steps, A.step0, A.resample, wc,
                                      tape + (seg & 1) * buf_stride, tape_step, lb);
            } else {
                const int seg = n_seg_all - t;
                if (t > 0 && seg < n_seg)
                    reverse_segment(c, lim, g, A.ckpt, ld, bo, A.K, seg, steps, A.step0, A.resample, wc,
                                    tape + (seg & 1) * buf_stride, tape_step, lb, lam, gk);
            }
            __syncthreads();
        }
        if (!producer && valid) {
            store_adj(A.grad_x0, A.grad_mem, ld, bo, lam);
            if (A.grad_gains) {
#pragma unroll
                for (int k = 0; k < 9; ++k) elem(A.grad_gains + k * ld, bo) = gk[k];
            }
        }
    }
}

/* ---- processing order by type: block histograms, scan, stable scatter ---- */

__global__ void __launch_bounds__(kOrderBlock) k_block_hist(const uint8_t* type, int64_t n, int n_types,
                                                            const int32_t* rank,
                                                            int32_t* counts /* [rank][nb] */) {
    __shared__ int32_t h[256];
    for (int t = threadIdx.x; t < n_types; t += blockDim.x) h[t] = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kOrderBlock + threadIdx.x;
    if (i < n) atomicAdd(&h[type_entry(type, (uint32_t)i, n_types)], 1);
    __syncthreads();
    for (int t = threadIdx.x; t < n_types; t += blockDim.x)
        counts[(int64_t)rank[t] * gridDim.x + blockIdx.x] = h[t];
}

/* Stable scatter: agent i of block b, type t, goes to base[rank t][b] plus
 * the number of earlier agents of type t in the block.  base is the
 * exclusive prefix sum of the counts laid out rank-major, i.e. the agents of
 * all lower-ranked types plus those of type t in earlier blocks. */
__global__ void __launch_bounds__(kOrderBlock) k_scatter(const uint8_t* type, int64_t n, int n_types,
                                                         const int32_t* rank, const int32_t* base, int32_t* perm) {
    __shared__ uint8_t ty[kOrderBlock];
    const int64_t i = (int64_t)blockIdx.x * kOrderBlock + threadIdx.x;
    const uint8_t mine = i < n ? (uint8_t)type_entry(type, (uint32_t)i, n_types) : 0;
    ty[threadIdx.x] = mine;
    __syncthreads();
    if (i >= n) return;
    int32_t before = 0;
    for (int j = 0; j < (int)threadIdx.x; ++j) before += ty[j] == mine ? 1 : 0;
    perm[base[(int64_t)rank[mine] * gridDim.x + blockIdx.x] + before] = (int32_t)i;
}

/* Agents whose first n_rows state rows hold a NaN or an infinity: one
 * count per wave (ballot), one atomic per wave. */
__global__ void __launch_bounds__(256) k_count_nonfinite(const float* rows, int64_t ld, int64_t n, int n_rows,
                                                         unsigned long long* count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (i < n) {
        const uint32_t bo = (uint32_t)i << 2;
        for (int k = 0; k < n_rows; ++k) bad |= !isfinite(elem(uniform(rows + k * ld), bo));
    }
    const unsigned long long mask = __ballot(bad);
    if (mask && (threadIdx.x & (warpSize - 1)) == (unsigned)(__ffsll((long long)mask) - 1))
        atomicAdd(count, (unsigned long long)__popcll(mask));
}

template <int MODE, bool HET, bool GAINS, bool CKPT, bool PERM, bool CARRY, bool KINDS>
const void* kfn() {
    return reinterpret_cast<const void*>(&k_rollout<MODE, HET, GAINS, CKPT, PERM, CARRY, KINDS>);
}

/* Checkpoints are only written with carries and only for quadrotor tables
 * (the host refuses the other combinations), so a variant with ckpt maps to
 * the checkpointing kernel, which reads and writes the carries. */
template <int MODE, bool HET, bool GAINS, bool PERM>
const void* kfn_carry(const Variant& v) {
    if (MODE == 1 && v.ckpt) return kfn<MODE, HET, GAINS, MODE == 1, PERM, true, false>();
    if (v.kinds)
        return v.carry ? kfn<MODE, HET, GAINS, false, PERM, true, true>()
                       : kfn<MODE, HET, GAINS, false, PERM, false, true>();
    return v.carry ? kfn<MODE, HET, GAINS, false, PERM, true, false>()
                   : kfn<MODE, HET, GAINS, false, PERM, false, false>();
}

}  // namespace

const void* rollout_kernel(const Variant& v) {
    /* open loop: gains and checkpoints do not apply */
    if (v.mode == 0) {
        if (!v.het) return kfn_carry<0, false, false, false>(v);
        return v.perm ? kfn_carry<0, true, false, true>(v) : kfn_carry<0, true, false, false>(v);
    }
#define POTATO_PICK(H, P) return v.gains ? kfn_carry<1, H, true, P>(v) : kfn_carry<1, H, false, P>(v);
    if (!v.het) { POTATO_PICK(false, false) }
    if (v.perm) { POTATO_PICK(true, true) }
    POTATO_PICK(true, false)
#undef POTATO_PICK
}

template <bool H, bool G, bool P>
const void* afn() {
    return reinterpret_cast<const void*>(&k_adjoint<H, G, P>);
}
template <bool H, bool G, bool P>
const void* apfn() {
    return reinterpret_cast<const void*>(&k_adjoint_pipe<H, G, P>);
}

size_t adjoint_lds_bytes(bool het, int n_types) {
    return ((sizeof(Limits) + 15) / 16) * 16 + (size_t)(het ? n_types : 1) * sizeof(TypeConst);
}

const void* adjoint_kernel(bool het, bool gains, bool perm, bool pipe) {
    if (pipe) {
        if (!het) return gains ? apfn<false, true, false>() : apfn<false, false, false>();
        if (perm) return gains ? apfn<true, true, true>() : apfn<true, false, true>();
        return gains ? apfn<true, true, false>() : apfn<true, false, false>();
    }
    if (!het) return gains ? afn<false, true, false>() : afn<false, false, false>();
    if (perm) return gains ? afn<true, true, true>() : afn<true, false, true>();
    return gains ? afn<true, true, false>() : afn<true, false, false>();
}

hipError_t launch_adjoint(bool het, bool gains, bool perm, bool pipe, const AdjArgs& a, int grid_blocks,
                          hipStream_t stream) {
    void* args[] = {const_cast<AdjArgs*>(&a)};
    const size_t lds = adjoint_lds_bytes(het, a.n_types);
    return hipLaunchKernel(adjoint_kernel(het, gains, perm, pipe), dim3((unsigned)grid_blocks),
                           dim3((unsigned)(pipe ? kAdjPipeBlock : kAdjBlock)), args, lds, stream);
}

bool rollout_grouped(const Variant& v, const StepArgs& a) {
    return v.het && !v.perm && !v.ckpt && a.n_groups >= 2;
}

size_t rollout_lds_bytes(const Variant& v, const StepArgs& a, int block) {
    return ((sizeof(Limits) + 15) / 16) * 16 + (size_t)(v.het ? a.n_types : 1) * sizeof(TypeConst) +
           (rollout_grouped(v, a) ? (size_t)group_lds_words(block) * sizeof(int32_t) : 0);
}

/* Blocks of `block` threads the chip holds at once for kernel fn with lds
 * bytes of dynamic LDS: the occupancy per compute unit times the compute
 * units of the current device, cached per (device, kernel, block, lds). */
static hipError_t fill_blocks(const void* fn, int block, size_t lds, int* out) {
    static std::mutex mu;
    static std::map<std::tuple<int, const void*, int, size_t>, int> cache;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const auto key = std::make_tuple(dev, fn, block, lds);
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end()) {
        *out = it->second;
        return hipSuccess;
    }
    int per_cu = 0, n_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, lds);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    *out = cache[key] = std::max(1, per_cu * n_cu);
    return hipSuccess;
}

hipError_t launch_rollout(const Variant& v, const StepArgs& a, int block, int grid_blocks,
                          hipStream_t stream) {
    const void* fn = rollout_kernel(v);
    int64_t grid = grid_blocks > 0 ? grid_blocks : (a.n + block - 1) / block;
    const size_t lds = rollout_lds_bytes(v, a, block);
    if (grid_blocks <= 0 && rollout_grouped(v, a)) {
        /* agents grouped per block: one round of blocks, as many as the
         * chip holds at once, so that each sorts chunks as wide as the
         * swarm allows */
        int fill = 0;
        hipError_t e = fill_blocks(fn, block, lds, &fill);
        if (e != hipSuccess) return e;
        grid = std::min<int64_t>(grid, fill);
    }
    if (grid > 0x7fffffff) grid = 0x7fffffff;
    void* args[] = {const_cast<StepArgs*>(&a)};
    return hipLaunchKernel(fn, dim3((unsigned)grid), dim3((unsigned)block), args, lds, stream);
}

hipError_t launch_count_nonfinite(const float* rows, int64_t ld, int64_t n, int n_rows, unsigned long long* count,
                                  hipStream_t stream) {
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_count_nonfinite, dim3(nb), dim3(256), 0, stream, rows, ld, n, n_rows, count);
    return hipGetLastError();
}

int64_t order_workspace_words(int64_t n, int n_types) {
    const int64_t m = ((n + kOrderBlock - 1) / kOrderBlock) * n_types;
    return 2 * m + scan_chunks((uint32_t)m) + 1;
}

hipError_t launch_order_by_type(const uint8_t* type, int64_t n, int n_types, const int32_t* rank,
                                int32_t* perm, int32_t* workspace, hipStream_t stream) {
    const int nb = (int)((n + kOrderBlock - 1) / kOrderBlock);
    const uint32_t m = (uint32_t)nb * (uint32_t)n_types;
    int32_t* counts = workspace;          /* [rank][nb] */
    int32_t* base = counts + m;           /* its exclusive prefix sum */
    int32_t* totals = base + m;           /* scan_chunks(m) chunk totals, then the grand total */
    hipLaunchKernelGGL(k_block_hist, dim3(nb), dim3(kOrderBlock), 0, stream, type, n, n_types, rank, counts);
    launch_exclusive_scan(counts, base, totals, totals + scan_chunks(m), m, stream);
    hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(kOrderBlock), 0, stream, type, n, n_types, rank, base, perm);
    return hipGetLastError();
}

}  // namespace potato
