/*
 * potato.h -- C ABI of the MI355X batched quadrotor simulator.
 *
 * The library advances N independent nonlinear quadrotors held as
 * structure-of-arrays FP32 device buffers.  One time step of one agent is:
 *   1. controller (closed loop): position -> attitude -> body-rate PID
 *      cascade whose innermost loop is the body-rate PID of Sec. II-B, then
 *      the mixer, which solves the allocation of eq. (3) for the four rotor
 *      thrusts, saturates them and inverts the rotor model of eq. (2);
 *      open loop instead holds caller-given rotor-speed commands;
 *   2. classical fourth-order Runge-Kutta over the rigid-body model of
 *      eqs. (qd1)-(qd4) (Sec. II-B), with rotor thrust and torque
 *      k_f W^2, k_m W^2 (eq. 2), first-order rotor lag and linear drag,
 *      the command held through the four stages;
 *   3. renormalisation of the attitude quaternion.
 * Batching homogeneous agents in tensors is the data-oriented design of
 * Sec. I (Fig. 1); several airframe types in one batch through a
 * per-agent type index replace the paper's one-process-per-type scheme.
 *
 * Conventions shared by every entry point:
 *   - All pointers named "device" are HIP device pointers owned by the
 *     caller; the library never frees them and never keeps them after the
 *     call returns (except inside a cached hipGraph, see potato_options).
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = default stream)
 *     and the call returns without synchronising.
 *   - Host-detectable errors return a status with no side effect and no
 *     work enqueued; launch failures return POTATO_EHIP.  The message of the
 *     last failure on the calling thread is potato_last_error().
 *   - No C++ exception crosses this interface.
 *
 * State layout: float32 rows[30][ld], one column per agent (ld >= n_agents):
 *   0-2 position (ENU inertial, m)      3-5 velocity (m/s)
 *   6-9 quaternion w,x,y,z (body FLU -> inertial, Hamilton product)
 *   10-12 body rates (rad/s)
 *   13-16 rotor speeds minus the type's w_ref (rad/s); rotors are numbered
 *         front-left, front-right, back-right, back-left; 1 and 3 give
 *         positive yaw reaction torque
 *   17-19 position-loop integral   20-22 attitude-loop integral
 *   23-25 rate-loop integral       26-28 body rates at the previous step
 *   29 running cost J = time integral of the sum of squared rotor speeds
 * Rows 0-16 are the rigid body and rotors of eqs. (qd1)-(qd4) and (2),
 * rows 17-28 the controller's memory.  Open-loop mode reads and writes rows
 * 0-16 only.  No call writes past row 29 of a state.
 *
 * Rounding carries (optional): float32 carry[10][carry_ld], one column per
 * agent (carry_ld >= n_agents): 0-2 position, 3-5 velocity, 6 J, 7-9
 * position-loop integral (cars and fixed-wing aircraft: row k holds the
 * carry of state row k, k = 0-6).  Each holds the low-order part that an FP32
 * update of its row dropped (compensated summation, Dekker's Fast2Sum), so
 * the represented value is row + carry; a fresh state has carries 0 and
 * they stay below one ulp of their row.  With a carry buffer the
 * integrator keeps them across calls and launches; without one (NULL) the
 * same arithmetic runs uncompensated.  Measured against the FP64 oracle on
 * the closed-loop swarm in a 100 m box (positions ~50 m, increments ~2 mm
 * per step, all rounded the same way): with carries the worst relative
 * state error is ~1e-6 after 1,000 and ~3e-6 after 10,000 steps; without,
 * ~1e-4 after 1,000 and ~2e-3 after 10,000 steps (the position's rounding
 * drift, fed back through the controller, shows in the body rates).
 */
#ifndef POTATO_H
#define POTATO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct potato_ctx potato_ctx;

typedef enum {
    POTATO_OK = 0,
    POTATO_EINVAL = 1,       /* invalid argument (nothing was enqueued) */
    POTATO_ENOMEM = 2,       /* host or device allocation failed */
    POTATO_EHIP = 3,         /* HIP runtime or launch failure */
    POTATO_EUNSUPPORTED = 4  /* valid but not implemented combination */
} potato_status;

enum { POTATO_OPEN_LOOP = 0, POTATO_CLOSED_LOOP = 1 };
enum { POTATO_FORM_AUTO = 0, POTATO_FORM_PLAIN = 1, POTATO_FORM_FUSED = 2 };
/* State rows, carry rows, checkpoint rows (a state and its carries). */
enum { POTATO_ROWS = 30, POTATO_CARRY_ROWS = 10, POTATO_CKPT_ROWS = 40 };
enum { POTATO_GAINS = 9, POTATO_MAX_TYPES = 256 };

/* One agent type (all FP32, SI units, angles in radians).
 *
 * kind POTATO_KIND_QUAD (0), the quadrotor of Sec. II-B: alpha is the
 * rotor-arm angle of the allocation matrix of eq. (3) (pi/4 for an X frame);
 * k_f, k_m are the thrust and torque coefficients of eq. (2) in
 * N/(rad/s)^2 and N m/(rad/s)^2; tau_m the rotor time constant (s); drag
 * the linear drag coefficient (N s/m); w_max the rotor speed limit (rad/s);
 * w_ref the reference speed the stored rotor rows are relative to (any
 * value; the hover speed keeps them small).  gains = [kpp kip kdp kpa kia
 * kda kpr kir kdr] (position, attitude, rate loops; P, I, D).  veh unused.
 *
 * kinds POTATO_KIND_CAR (1) and POTATO_KIND_WING (2), the two other robot
 * kinds of Sec. II-B: a car on the kinematic bicycle model and a
 * fixed-wing aircraft on the coordinated-turn guidance model, both guided
 * in closed loop around an orbit of radius rho about their waypoint
 * (circle trajectories as in the first demonstration of Sec. IV).  Only
 * mass, drag (car: longitudinal, N s/m), radius, step_budget, kind and
 * veh are read:
 *   car:  veh = [L wheelbase (m), l_r centre of mass to rear axle (m),
 *                tau_delta steering lag (s), delta_max (rad),
 *                a_max (m/s^2), v_cruise (m/s), rho (m), lambda (+1
 *                counter-clockwise, -1 clockwise), k_orb, k_head, k_speed];
 *         needs L, tau_delta, rho > 0 and rho > l_r.
 *   wing: veh = [tau_V, tau_phi, tau_gamma (s), phi_max, gamma_max (rad),
 *                V_cruise (m/s), rho (m), lambda, k_orb, k_head, k_alt];
 *         needs the time constants, V_cruise and rho > 0.
 * Their state rows and inputs are listed at potato_step.
 *
 * Every kind: radius is the collision radius (m) used by
 * potato_detect_collisions; step_budget: an agent of this type is advanced
 * only while its global step index is below it (INT32_MAX = unlimited). */
enum { POTATO_KIND_QUAD = 0, POTATO_KIND_CAR = 1, POTATO_KIND_WING = 2 };
typedef struct {
    float mass, Ixx, Iyy, Izz, arm, alpha, k_f, k_m, tau_m, drag, w_max, w_ref, radius;
    float gains[9];
    int32_t step_budget;
    int32_t kind;
    float veh[12];
} potato_type_params;

/* Controller limits shared by all types: gravity g, position-error
 * saturation radius r_sat (m), integral clamps, and the lower bound of the
 * commanded vertical acceleration as a fraction of g. */
typedef struct {
    float g, r_sat, ipos_max, iatt_max, irate_max, az_min_frac;
} potato_limits;

/* Launch policy.  form: plain = one launch per time step (state round-trips
 * through HBM every step); fused = steps_per_launch steps per launch with
 * the state in registers; auto = fused.  block / steps_per_launch /
 * grid_blocks = 0 select the tuned value (potato_autotune) or a default.
 * use_graph != 0 captures the launches of a potato_step call in a hipGraph
 * cached on the context and replays it when the same call (same pointers,
 * sizes, step index and time step) is made again. */
typedef struct {
    int32_t mode;              /* POTATO_OPEN_LOOP or POTATO_CLOSED_LOOP */
    int32_t form;              /* POTATO_FORM_* */
    int32_t block;             /* threads per block: 64, 128, 256, 512, 1024 or 0 */
    int32_t steps_per_launch;  /* fused form, >= 1 or 0 */
    int32_t grid_blocks;       /* fused form: blocks in the grid-stride loop, 0 = one agent per thread */
    int32_t use_graph;
} potato_options;

/* Device state rows[30][ld] (in place) and its optional rounding carries
 * carry[10][carry_ld] (in place; NULL: uncompensated updates, carry_ld is
 * then ignored). */
typedef struct {
    float* rows;
    int64_t ld;
    float* carry;
    int64_t carry_ld;
} potato_state;

/* Optional per-agent data (device pointers; each may be NULL):
 *   type   uint8[n_agents] type index into the context's table (NULL: all
 *          type 0).  The device reads a value >= n_types as n_types - 1
 *          (it does not report it; the Python binding's debug mode does).
 *   perm   int32[n_agents] processing order: lane j advances agent perm[j]
 *          (a permutation of 0..n_agents-1, e.g. from
 *          potato_order_by_type).  NULL = identity.  The device reads an
 *          entry outside [0, n_agents) as n_agents - 1: nothing outside the
 *          rows is addressed, but an order that is not a permutation leaves
 *          agents unadvanced and races on others.  Without an order, a
 *          launch whose types fall into 2 to 8 classes of equal step budget
 *          and kind groups each block's agents by class itself (the same
 *          results, bit for bit; with more classes, pass the order for
 *          waves of one budget and kind).
 *   gains  float[9][gains_ld] per-agent gains (NULL: the type's gains).
 *   alive  uint8[n_agents]: agents with 0 are dead and are neither advanced
 *          nor differentiated (their state and cotangent pass through);
 *          NULL: all alive.  potato_detect_collisions maintains it. */
typedef struct {
    const uint8_t* type;
    const int32_t* perm;
    const float* gains;
    int64_t gains_ld;
    const uint8_t* alive;
} potato_params;

/* Commands (device pointers):
 *   motor_cmd float[4][ld] open-loop rotor commands relative to w_ref,
 *             held for the whole call;
 *   wp        float[n_epochs][3][ld] closed-loop waypoints; the step with
 *             global index k uses epoch min(k / resample_every, n_epochs-1)
 *             (resample_every <= 0: epoch 0);
 *   step0     global index of the first step of the call (for the waypoint
 *             epoch and the step budget). */
typedef struct {
    const float* motor_cmd;
    const float* wp;
    int32_t n_epochs;
    int32_t resample_every;
    int64_t ld;
    int64_t step0;
} potato_cmds;

/* Create a context for `n_types` airframe types (1..256).  Validates the
 * table (positive mass, inertia, arm, k_f, k_m, tau_m; finite values),
 * derives per-type constants once on the host (in double, rounded to FP32;
 * all per-agent arithmetic on the device is FP32) and copies the table to
 * the current HIP device.  *out is NULL on failure. */
potato_status potato_create(potato_ctx** out, const potato_type_params* types, int32_t n_types,
                            const potato_limits* limits, const potato_options* opts);

/* Release the context, its device table and cached graphs.  NULL is a no-op. */
potato_status potato_destroy(potato_ctx* ctx);

/* Replace the launch policy (also drops cached graphs). */
potato_status potato_set_options(potato_ctx* ctx, const potato_options* opts);

/*
 * Advance agents 0..n_agents-1 by n_steps time steps of length dt in place.
 * An agent of type t takes min(n_steps, max(0, step_budget_t - step0))
 * steps.  Cars and fixed-wing aircraft (types of kind 1 and 2) use rows 0-6
 * of the state: 0-2 position, 3 speed (m/s), 4 heading (car yaw, aircraft
 * course; from +x towards +y), 5 steering angle (car) or bank angle
 * (aircraft, positive turns left), 6 flight-path angle (aircraft); they do
 * not touch rows 7-29, nor a car rows 2 and 6 (nor those carry rows); for
 * them carry row k (k = 0-6) holds the rounding carry of state row k.  Their open-loop inputs are motor_cmd rows 0-2
 * (car: acceleration, steering command; aircraft: airspeed, bank and
 * flight-path commands), held for the call; in closed loop their waypoint
 * is the centre of the orbit they fly.  Errors (POTATO_EINVAL): ctx/state/params/cmds NULL, rows NULL,
 * n_agents outside [1, 2^30], ld < n_agents, carry given with carry_ld <
 * n_agents, n_steps < 0, dt not finite and > 0, missing motor_cmd (open
 * loop) or wp / n_epochs < 1 (closed loop), cmds->ld < n_agents, gains_ld <
 * n_agents when gains are given, ckpt set with ckpt_every < 1 or without a
 * carry buffer.  POTATO_EUNSUPPORTED: ckpt with a type table that holds
 * cars or fixed-wing aircraft (the adjoint covers quadrotors).  n_steps == 0
 * is a no-op.
 * ckpt (optional, device float[ceil(n_steps/ckpt_every)][40][ld]): slot c
 * receives the state (rows 0-29) and its carries (rows 30-39) at
 * call-relative step c*ckpt_every, before that step; it is what
 * potato_step_backward consumes, whose recomputation replays the
 * compensated integrator (hence the carry buffer).  Requires the fused form.
 */
potato_status potato_step(potato_ctx* ctx, const potato_state* state, const potato_params* params,
                          const potato_cmds* cmds, float dt, int64_t n_agents, int32_t n_steps,
                          float* ckpt, int32_t ckpt_every, void* stream);

/*
 * Time the fused form over a grid of (block in {64, 128, 256, 512, 1024}, steps
 * per launch in {25, 50, 100, 200, 500, 1000} up to probe_steps, grid of one
 * agent per thread or 1x / 2x the resident blocks) on a scratch copy of the
 * given inputs (the caller's buffers are not modified), store the fastest on
 * the context for this mode, type layout and checkpointing, and return it
 * in *best (may be NULL).  probe_steps is the number of time steps per
 * timed trial.  ckpt_every > 0 times the variant that writes checkpoints
 * every ckpt_every steps (into scratch memory), which potato_step runs when
 * given a checkpoint buffer; its result applies to such calls, 0 times and
 * tunes the variant without.  Errors as potato_step with the same
 * arguments; POTATO_EINVAL for ckpt_every < 0.  Allocates scratch memory
 * for the duration of the call and synchronises `stream`.
 */
potato_status potato_autotune(potato_ctx* ctx, const potato_state* state, const potato_params* params,
                              const potato_cmds* cmds, float dt, int64_t n_agents, int32_t probe_steps,
                              int32_t ckpt_every, potato_options* best, void* stream);

/*
 * Build a processing order for heterogeneous batches: perm (device
 * int32[n_agents]) lists agents grouped by type, types ordered by step
 * budget (longest first, ties by type index), agents of one type in
 * increasing index order.  Waves then hold one type and the longest
 * budgets are scheduled first.  type (device uint8[n_agents]): values
 * >= n_types are read as n_types - 1.  workspace: device buffer of at least
 * potato_order_workspace_bytes(n_agents, n_types) bytes.
 */
int64_t potato_order_workspace_bytes(int64_t n_agents, int32_t n_types);
potato_status potato_order_by_type(potato_ctx* ctx, const uint8_t* type, int64_t n_agents,
                                   int32_t* perm, void* workspace, int64_t workspace_bytes,
                                   void* stream);

/*
 * Reverse mode of a closed-loop potato_step call that wrote checkpoints:
 * given grad_final = dL/dx_N (device float[30][ld], the 30 rows of the
 * final state), compute grad_x0 = dL/dx_0 for the initial rigid-body and
 * rotor state (device float[17][ld]: rows 0-16 of the state layout), if
 * grad_mem is not NULL the cotangent of the initial controller memory and
 * cost (device float[13][ld]: state rows 17-29), and, if grad_gains is not
 * NULL, dL/dgains per agent (device float[9][ld]; with type gains the
 * caller sums over the agents of a type).  This is the vector-Jacobian
 * product of the rollout map (x_0, gains) -> x_N through every step of the
 * forward pass: controller, mixer, RK4 stages and renormalisation (the time
 * discretisation of Sec. II-B differentiated exactly, not the continuous
 * adjoint).  A carry has the cotangent of its row.
 *   params, cmds, dt, n_agents, n_steps: exactly as in the forward call;
 *   ckpt, ckpt_every: the checkpoints that call wrote (40 rows per slot:
 *   the state and its carries);
 *   workspace: device scratch of potato_backward_workspace_bytes() bytes
 *   (per-thread recomputation tape of ckpt_every steps).
 * Each segment of ckpt_every steps is recomputed from its checkpoint, then
 * reversed; for swarms too small to give every SIMD two waves, one wave
 * recomputes the next segment while another reverses the current one, with
 * the same result bit for bit.  Errors: POTATO_EINVAL as in potato_step, plus null ckpt,
 * grad_final or grad_x0, ckpt_every < 1 or a workspace that is too small;
 * POTATO_EUNSUPPORTED in open-loop mode and for a context whose type table
 * holds cars or fixed-wing aircraft.  grad_x0 may alias rows 0-16 of
 * grad_final and grad_mem rows 17-29 (each agent's column is read before
 * it is written).
 */
int64_t potato_backward_workspace_bytes(potato_ctx* ctx, const potato_params* params, int64_t n_agents,
                                        int32_t ckpt_every);
potato_status potato_step_backward(potato_ctx* ctx, const potato_params* params, const potato_cmds* cmds,
                                   float dt, int64_t n_agents, int32_t n_steps, const float* ckpt,
                                   int32_t ckpt_every, int64_t ld, const float* grad_final,
                                   float* grad_x0, float* grad_mem, float* grad_gains, void* workspace,
                                   int64_t workspace_bytes, void* stream);

/*
 * Collision detection (the detection module of Sec. II-A: colliding agents
 * are marked dead and excluded).  Among agents with alive[i] != 0 on entry,
 * every agent i for which some other such agent j satisfies
 * |p_i - p_j|^2 < (r_i + r_j)^2 gets alive[i] = 0; r is the type's radius.
 * The test is FP32 with the operation order d2 = (dx*dx + dy*dy) + dz*dz,
 * dx = x_i - x_j, compared against (r_i + r_j)*(r_i + r_j), no contraction;
 * positions are rows 0-2 of the state.  All decisions use the entry alive
 * set.  alive: device uint8[n_agents], in/out.  died (device int64, may be
 * NULL) is incremented by the number of agents marked dead.  params->type is
 * the optional type index; other params fields are ignored.  Exact for
 * |coordinates| below 2^16 cell edges (cell edge 2.02 r_max; 22 km at
 * r = 0.17 m).  workspace: potato_collision_workspace_bytes(n_agents) bytes.
 */
int64_t potato_collision_workspace_bytes(int64_t n_agents);
potato_status potato_detect_collisions(potato_ctx* ctx, const potato_state* state, const potato_params* params,
                                       int64_t n_agents, uint8_t* alive, int64_t* died, void* workspace,
                                       int64_t workspace_bytes, void* stream);

/*
 * potato_detect_collisions without a caller workspace, for callers that
 * cannot allocate device memory (code under hipGraph capture, serving loops
 * with a fixed memory budget, harnesses that forbid hipMalloc).  Same
 * arguments, decisions and errors as potato_detect_collisions, but the
 * pass's scratch memory (the positions in partition and in bucket order,
 * the bucket starts, the partition offsets) is a static device array of the
 * library, sized for POTATO_NOALLOC_MAX_AGENTS agents (about 90 MiB, held
 * by every GPU the library runs on until the process ends); the call
 * allocates nothing.
 * Errors: POTATO_EINVAL as in potato_detect_collisions, and for
 * n_agents > POTATO_NOALLOC_MAX_AGENTS.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (other streams, other host
 * threads, other contexts) race and must be serialised by the caller;
 * calls on one stream are ordered and safe.
 */
enum { POTATO_NOALLOC_MAX_AGENTS = 1 << 20 };
potato_status potato_detect_collisions_noalloc(potato_ctx* ctx, const potato_state* state,
                                               const potato_params* params, int64_t n_agents, uint8_t* alive,
                                               int64_t* died, void* stream);

/*
 * Command ingress and snapshot egress around a running rollout (Sec. II-A,
 * Fig. 2: the decision side is kept out of the simulation loop, so the
 * simulated world keeps running while new commands are produced, and the
 * states are streamed out to a viewer).  A pipe owns two device command
 * slots, two device position slots, a pinned host staging copy of each
 * command slot and two copy streams (ingress and egress), all allocated by
 * potato_pipe_create, so runs and pushes allocate nothing.
 *
 *   potato_pipe_push(pipe, host_cmd): host_cmd is host memory (any kind)
 *     float[rows][n_agents], rows = 3 (closed loop: waypoint x, y, z) or
 *     4 (open loop: rotor commands relative to w_ref).  It is copied into
 *     the pinned staging slot before the call returns (the caller may
 *     reuse it at once), then to the device slot on the ingress stream,
 *     after the runs that read that slot's previous contents.  Blocks the
 *     host only while the same staging slot's previous upload is still in
 *     flight (two pushes ahead of the GPU).
 *   potato_pipe_run(pipe, state, params, dt, n_steps, snap_every,
 *     host_snap, stream): advances state (as potato_step with the
 *     context's launch options, without graph capture) by n_steps with
 *     the most recently pushed commands (held for the whole run; the
 *     stream waits for their upload).  The
 *     pipe keeps the global step index across runs (step budgets).  With
 *     snap_every > 0, after every snap_every steps the positions (rows
 *     0-2) go to host_snap[k] (float[n_steps / snap_every][3][n_agents],
 *     host memory).  Pinned memory from hipHostMalloc (what torch's
 *     pin_memory gives) is written directly by the last launch before the
 *     snapshot, as its waves finish, so the transfer overlaps the rest of
 *     that launch; any other host memory goes through a device slot and a
 *     download on the egress stream.  Snapshot k of the run holds the
 *     positions after step (k+1)*snap_every of the run; host_snap must
 *     stay allocated, and unread, until potato_pipe_wait_snapshots (or
 *     potato_pipe_sync) reports the snapshot landed.  Every run of a pipe
 *     must use the same stream.
 *   potato_pipe_stats(pipe, snapshots, direct): snapshots enqueued since
 *     creation, and how many of them were written directly to pinned host
 *     memory.
 *   potato_pipe_wait_snapshots(pipe, count): blocks until the first
 *     `count` snapshots taken by the pipe since its creation (counted over
 *     all runs) are in host memory.
 *   potato_pipe_sync(pipe): blocks until all enqueued uploads and
 *     snapshots are done.
 *   potato_pipe_destroy(pipe): synchronises the pipe's streams and the run
 *     stream, then frees the pipe.  NULL is a no-op.  Destroy a pipe before
 *     its context and before the stream its runs used.
 * A pipe is not thread-safe: one host thread drives it.
 * Errors: POTATO_EINVAL for null pointers, n_agents < 1, a run before the
 * first push, n_steps < 0, snap_every < 0, missing host_snap when a
 * snapshot is due, a pinned host_snap whose allocation ends before the
 * snapshots due, a run on another stream than the first run, or a
 * context whose mode changed since the pipe was created; the errors of
 * potato_step otherwise.  After a POTATO_EHIP the pipe must be destroyed.
 */
typedef struct potato_pipe potato_pipe;
potato_status potato_pipe_create(potato_ctx* ctx, int64_t n_agents, potato_pipe** out);
potato_status potato_pipe_push(potato_pipe* pipe, const float* host_cmd);
potato_status potato_pipe_run(potato_pipe* pipe, const potato_state* state, const potato_params* params,
                              float dt, int32_t n_steps, int32_t snap_every, float* host_snap, void* stream);
potato_status potato_pipe_wait_snapshots(potato_pipe* pipe, int64_t count);
potato_status potato_pipe_sync(potato_pipe* pipe);
potato_status potato_pipe_stats(const potato_pipe* pipe, int64_t* snapshots, int64_t* direct);
potato_status potato_pipe_destroy(potato_pipe* pipe);

/*
 * Failure detection: adds to *count (device int64) the number of agents
 * 0..n_agents-1 whose state holds a NaN or an infinity in the rows the
 * context's mode integrates (closed loop: rows 0-29, open loop: rows 0-16).
 * Agents are independent, so a non-finite agent never contaminates another
 * (the count is the number of diverged agents, not a global flag).
 * Errors: POTATO_EINVAL for null pointers, n_agents outside [1, 2^30] or
 * state.ld < n_agents.
 */
potato_status potato_count_nonfinite(potato_ctx* ctx, const potato_state* state, int64_t n_agents, int64_t* count,
                                     void* stream);

/* Message of the last failed call on the calling thread ("" if none),
 * valid until that thread's next call into the library.  ctx may be NULL
 * (failures of potato_create and of calls without a context are recorded
 * the same way); the message is per thread, not per context. */
const char* potato_last_error(const potato_ctx* ctx);

/* Library version string. */
const char* potato_version(void);

#ifdef __cplusplus
}
#endif

#endif /* POTATO_H */
