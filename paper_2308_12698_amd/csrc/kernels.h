/*
 * kernels.h -- internal interface between the C ABI (abi.hip) and the
 * gfx950 kernels (kernels.hip).  Not installed; not part of the ABI.
 */
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "quad_step.h"

namespace potato {

constexpr int kRows = 30;       /* state rows per agent, see include/potato.h */
constexpr int kCarryRows = 10;  /* rounding-carry rows per agent */
constexpr int kCkptRows = 40;   /* checkpoint slot: the state, then its carries */

/* Largest agent count: agent index times 4 (a byte offset into a row) must
 * fit 32 bits, which the kernels' row addressing relies on. */
constexpr int64_t kMaxAgents = int64_t(1) << 30;

/* Everything one rollout launch needs, passed by value as the kernel
 * argument (uniform, lands in scalar registers). */
struct StepArgs {
    float* rows;                 /* [kRows][ld] */
    int64_t ld;
    float* carry;                /* [kCarryRows][carry_ld] or null (uncompensated) */
    int64_t carry_ld;
    int64_t n;                   /* agents (lanes) */
    const uint8_t* type;         /* [ld] or null */
    const int32_t* perm;         /* [n] or null */
    const float* gains;          /* [9][gains_ld] or null */
    int64_t gains_ld;
    const float* motor_cmd;      /* [4][cmd_ld] */
    const float* wp;             /* [n_epochs][3][cmd_ld] */
    int64_t cmd_ld;
    int32_t n_epochs;
    int32_t resample;
    int64_t step0;               /* global index of this launch's first step */
    int32_t n_steps;             /* steps in this launch */
    int32_t k0;                  /* call-relative index of this launch's first step */
    float* ckpt;                 /* [slots][kCkptRows][ld] or null (needs carry) */
    int32_t ckpt_every;
    int32_t n_types;
    const TypeConst* table;      /* device [n_types] */
    const uint8_t* alive;        /* [ld] or null: 0 = dead, not advanced */
    int32_t n_groups;            /* classes of types grouped within a block (a per-agent
                                    type and no processing order), or 0: none */
    float* snap;                 /* [3][n] device view of pinned host memory, or null: every
                                    agent's position after this launch (not with ckpt) */
    Limits lim;
};

struct Variant {
    int mode;        /* 0 open loop, 1 closed loop */
    bool het;        /* per-agent type index, LDS table */
    bool gains;      /* per-agent gains */
    bool ckpt;       /* write checkpoints */
    bool perm;       /* processing order */
    bool carry;      /* rounding carries kept in a carry buffer */
    bool kinds;      /* the type table holds cars or fixed-wing aircraft */
};

/* Arguments of the adjoint (reverse sweep) launch. */
struct AdjArgs {
    const float* ckpt;           /* [slots][kCkptRows][ld] from the forward call */
    int64_t ld;
    int64_t n;
    const uint8_t* type;
    const int32_t* perm;
    const float* gains;
    int64_t gains_ld;
    const float* wp;
    int64_t cmd_ld;
    int32_t n_epochs;
    int32_t resample;
    int64_t step0;
    int32_t n_steps;
    int32_t K;                   /* checkpoint interval */
    const float* grad_final;     /* [30][ld] */
    float* grad_x0;              /* [17][ld]: rows 0-16 */
    float* grad_mem;             /* [13][ld] or null: rows 17-29 */
    float* grad_gains;           /* [9][ld] or null */
    float* tape;                 /* layouts at launch_adjoint */
    int64_t tape_ld;             /* threads in the grid (a multiple of 64) */
    int32_t n_types;
    const TypeConst* table;
    const uint8_t* alive;
    Limits lim;
};

/* Agents of a per-agent type in the caller's order (no checkpoints) are
 * stepped grouped by class (types of equal step budget and kind; 2 to
 * kMaxGroups classes) within chunks of up to kGroupWidths block widths.
 * Unless a grid is given, such a launch takes as many blocks as the chip
 * holds at once (fewer if the swarm needs fewer); each block owns
 * ceil(n / grid) agents, rounded up to a multiple of 64.  The sort takes
 * group_lds_words(block) words of LDS after the type table. */
constexpr int kGroupWidths = 4;
constexpr int kMaxGroups = 8;
__host__ __device__ constexpr int64_t group_lds_words(int block) {
    return 2 * (int64_t)kGroupWidths * (block / 64) * kMaxGroups + (int64_t)kGroupWidths * block +
           kMaxGroups * 64 + 2 * ((int64_t)kGroupWidths * (block / 64) + kMaxGroups) + 4 * kMaxGroups + 2;
}

/* Launch one rollout kernel (n_steps of args) on `stream`. */
hipError_t launch_rollout(const Variant& v, const StepArgs& a, int block, int grid_blocks,
                          hipStream_t stream);

/* Kernel function pointer of a variant (occupancy queries). */
const void* rollout_kernel(const Variant& v);

/* Adjoint: kernel pointer (occupancy queries) and launch of grid_blocks
 * blocks.  One agent per thread, kAdjBlock threads per block, tape
 * [K][grid threads / 64][kTapeRows][64]; or, with `pipe`, kAdjPipeBlock
 * threads per block serving 64 agents with one recomputing and one
 * reversing wave, tape [grid][2][K][kTapeRows][64].  Either way the tape
 * takes K x kTapeRows x grid x block floats. */
const void* adjoint_kernel(bool het, bool gains, bool perm, bool pipe);
hipError_t launch_adjoint(bool het, bool gains, bool perm, bool pipe, const AdjArgs& a, int grid_blocks,
                          hipStream_t stream);
size_t adjoint_lds_bytes(bool het, int n_types);
constexpr int kAdjBlock = 256;
constexpr int kAdjPipeBlock = 128;
/* Use the pipelined adjoint for small swarms (1) or never (0). */
#ifndef POTATO_ADJOINT_PIPE
#define POTATO_ADJOINT_PIPE 1
#endif

/* Dynamic LDS bytes of a launch: the limits, a.n_types type-table entries
 * and, when it groups its agents, the sort's words. */
size_t rollout_lds_bytes(const Variant& v, const StepArgs& a, int block);
bool rollout_grouped(const Variant& v, const StepArgs& a);

/* Processing order by type (see potato_order_by_type): workspace of
 * order_workspace_words(n, n_types) int32 words. */
int64_t order_workspace_words(int64_t n, int n_types);
hipError_t launch_order_by_type(const uint8_t* type, int64_t n, int n_types,
                                const int32_t* type_rank_dev, int32_t* perm,
                                int32_t* workspace, hipStream_t stream);

constexpr int kOrderBlock = 256;

/* Adds to *count the agents whose first n_rows rows hold a non-finite value. */
hipError_t launch_count_nonfinite(const float* rows, int64_t ld, int64_t n, int n_rows, unsigned long long* count,
                                  hipStream_t stream);

/* Collision detection on a hashed grid (see collide.hip). */
int64_t collision_workspace_bytes(int64_t n);
/* Largest swarm of the allocation-free collision entry point. */
constexpr int64_t kNoAllocMaxAgents = int64_t(1) << 20;
/* Device address (current device) and size of that entry point's static
 * workspace; the address is looked up once per device and kept. */
hipError_t collision_scratch(void** ptr, int64_t* bytes);
hipError_t launch_detect_collisions(const float* rows, int64_t ld, int64_t n, const uint8_t* type, int n_types,
                                    const float* radius_dev, float r_max, uint8_t* alive,
                                    unsigned long long* died, void* workspace, hipStream_t s);

}  // namespace potato
