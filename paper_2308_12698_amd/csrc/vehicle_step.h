/*
 * vehicle_step.h -- per-agent FP32 arithmetic of one time step of the two
 * other robot kinds the simulator batches with its quadrotors (the paper
 * names fixed-wing drones, quadrotors and cars, Sec. II-B, and writes out
 * only the quadrotor; the other two follow the works it cites for them):
 *   - car (kind 1): the kinematic bicycle model referenced at the centre of
 *     mass (Rajamani, Vehicle Dynamics and Control, 2nd ed., Sec. 2.2):
 *     side-slip beta = atan(l_r tan(delta) / L), position rate
 *     v (cos(psi + beta), sin(psi + beta)), yaw rate v cos(beta) tan(delta) / L,
 *     a first-order steering actuator and an acceleration input with
 *     linear drag;
 *   - fixed wing (kind 2): the kinematic guidance model of Beard and
 *     McLain (Small Unmanned Aircraft, Ch. 9) in still air: velocity V along
 *     course chi and flight-path angle gamma, coordinated-turn course rate
 *     g tan(phi) / V, first-order airspeed, roll and flight-path responses;
 *   - guidance of both in closed loop: the orbit-following vector field of
 *     the same book (Ch. 10) around the agent's waypoint, radius rho,
 *     direction lambda: course command
 *     atan2(y - c_y, x - c_x) + lambda (pi/2 + atan(k_orb (d - rho) / rho)),
 *     plus the steering or bank that holds the circle exactly, a speed hold
 *     (car) and a saturated altitude hold (aircraft).  These are the circle
 *     trajectories of the paper's first demonstration (Sec. IV).
 * State rows (of the simulator's [30][ld] layout; rows 7-29 are not
 * touched): 0-2 position, 3 speed, 4 heading (car yaw psi, aircraft course
 * chi), 5 actuator angle (steering delta, bank phi), 6 flight-path angle
 * gamma (aircraft only; a car leaves rows 2 and 6 unchanged).  Inputs, held
 * through the step: car (a_c, delta_c), aircraft (V_c, phi_c, gamma_c).
 *
 * Differences from a literal transcription, all exact in real arithmetic:
 * cos(beta) and sin(beta) are 1/sqrt(1 + t^2) and t/sqrt(1 + t^2) with
 * t = tan(beta), and cos/sin(psi + beta) are expanded by the angle-sum
 * formulas, so a car's derivative takes one tangent and one sine-cosine
 * pair instead of an arctangent and three trigonometric calls; divisions by
 * the time constants, the wheelbase and g rho are multiplications by
 * reciprocals precomputed per type; the car's steering feed-forward is a
 * per-type constant.  Every integrated row keeps a rounding carry
 * (Fast2Sum), as the quadrotor's position and velocity do.  Contraction is
 * off and fused multiply-adds are placed explicitly, so the plain and the
 * fused launches give the same bits.
 */
#pragma once

#include "quad_step.h"

namespace potato {

constexpr float kTwoPi = 6.28318530717958647692f;
constexpr float kInvTwoPi = 0.159154943091895335769f;

/* Angle a moved into [-pi, pi] by whole turns. */
__device__ __forceinline__ float wrap_pi(float a) {
    return POTATO_FMA(-kTwoPi, rintf(a * kInvTwoPi), a);
}

/* Rows a kind integrates (the car has no altitude or flight-path dynamics). */
template <int KIND>
__device__ __forceinline__ constexpr bool veh_row(int k) {
    return KIND == KIND_WING || (k != 2 && k != 6);
}

/* Rates of rows 0-6 at state x with inputs u held. */
template <int KIND>
__device__ __forceinline__ void veh_rates(const VehConst& c, const float x[7], const float u[3], float dx[7]) {
#pragma clang fp contract(off)
    float sh, ch;
    sincosf(x[4], &sh, &ch);
    if (KIND == KIND_CAR) {
        const float td = tanf(x[5]);
        const float tb = c.lr_L * td;                         /* tan(beta) */
        const float cb = rsq(POTATO_FMA(tb, tb, 1.0f));       /* cos(beta) > 0 */
        const float sb = tb * cb;                             /* sin(beta) */
        const float cc = POTATO_FMA(ch, cb, -(sh * sb));      /* cos(psi + beta) */
        const float sc = POTATO_FMA(sh, cb, ch * sb);         /* sin(psi + beta) */
        dx[0] = x[3] * cc;
        dx[1] = x[3] * sc;
        dx[2] = 0.0f;
        dx[3] = POTATO_FMA(-c.cd_m, x[3], u[0]);
        dx[4] = (x[3] * cb) * (td * c.inv_L);
        dx[5] = (u[1] - x[5]) * c.inv_tau[0];
        dx[6] = 0.0f;
    } else {
        float sg, cg;
        sincosf(x[6], &sg, &cg);
        const float vh = x[3] * cg;                           /* horizontal speed */
        dx[0] = vh * ch;
        dx[1] = vh * sh;
        dx[2] = x[3] * sg;
        dx[3] = (u[0] - x[3]) * c.inv_tau[0];
        dx[4] = (c.g * tanf(x[5])) / x[3];
        dx[5] = (u[1] - x[5]) * c.inv_tau[1];
        dx[6] = (u[2] - x[6]) * c.inv_tau[2];
    }
}

/* Closed-loop inputs from the step-start state x around orbit centre wp. */
template <int KIND>
__device__ __forceinline__ void veh_guidance(const VehConst& c, const float x[7], const float wp[3], float u[3]) {
#pragma clang fp contract(off)
    const float ex = x[0] - wp[0], ey = x[1] - wp[1];
    const float d = sqrtf(POTATO_FMA(ey, ey, ex * ex));
    const float chi_d = POTATO_FMA(c.lam, atanf(c.k_orb_rho * (d - c.rho)), atan2f(ey, ex) + c.lam_half_pi);
    if (KIND == KIND_CAR) {
        /* the car's course is its yaw plus the side-slip angle */
        const float beta = atanf(c.lr_L * tanf(x[5]));
        const float e = wrap_pi(chi_d - (x[4] + beta));
        u[0] = clampf_(POTATO_FMA(c.k_hold, c.cruise - x[3], c.cd_m * x[3]), -c.lim[0], c.lim[0]);
        u[1] = clampf_(POTATO_FMA(c.k_head, e, c.ff), -c.lim[1], c.lim[1]);
        u[2] = 0.0f;
    } else {
        /* bank that holds the circle: tan(phi) = V^2 / (g rho) */
        const float e = wrap_pi(chi_d - x[4]);
        const float ff = c.lam * atanf((x[3] * x[3]) * c.inv_g_rho);
        u[0] = c.cruise;
        u[1] = clampf_(POTATO_FMA(c.k_head, e, ff), -c.lim[1], c.lim[1]);
        u[2] = clampf_(c.k_hold * (wp[2] - x[2]), -c.lim[2], c.lim[2]);
    }
}

/* Classical RK4 over rows 0-6 with the inputs held; CARRY: every
 * integrated row keeps its rounding carry in lo (the heading matters most:
 * it grows by nearly equal increments every step, and a rounding bias of
 * its updates would be cancelled by a steady steering or bank offset). */
template <int KIND, bool CARRY>
__device__ __forceinline__ void veh_rk4(const VehConst& c, const Limits& L, float x[7], float lo[7],
                                        const float u[3]) {
#pragma clang fp contract(off)
    float k[7], acc[7], xs[7];
    veh_rates<KIND>(c, x, u, k);
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        acc[i] = k[i];
        xs[i] = veh_row<KIND>(i) ? POTATO_FMA(L.half_dt, k[i], x[i]) : x[i];
    }
    veh_rates<KIND>(c, xs, u, k);
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        acc[i] = POTATO_FMA(2.0f, k[i], acc[i]);
        xs[i] = veh_row<KIND>(i) ? POTATO_FMA(L.half_dt, k[i], x[i]) : x[i];
    }
    veh_rates<KIND>(c, xs, u, k);
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        acc[i] = POTATO_FMA(2.0f, k[i], acc[i]);
        xs[i] = veh_row<KIND>(i) ? POTATO_FMA(L.dt, k[i], x[i]) : x[i];
    }
    veh_rates<KIND>(c, xs, u, k);
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        if (!veh_row<KIND>(i)) continue;
        add_carry<CARRY>(x[i], lo[i], L.dt6 * (acc[i] + k[i]));
    }
}

}  // namespace potato
