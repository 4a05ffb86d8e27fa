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
 * Differences from a literal transcription, exact in real arithmetic or to
 * below FP32 rounding: cos(beta) and sin(beta) are 1/sqrt(1 + t^2) and
 * t/sqrt(1 + t^2) with t = tan(beta), and cos/sin(psi + beta) are expanded
 * by the angle-sum formulas, so a car's derivative takes no arctangent; the
 * trigonometric functions of the angles are evaluated once per step, at
 * the step-start state, and carried to each RK4 stage's angles by the
 * angle-sum formulas with short series for the stage's small offset
 * (sincos_shift, tan_shift); divisions by
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

/* Trigonometric functions of the angles of a state: heading (sh, ch),
 * tangent of the actuator angle (ta), flight-path angle (sg, cg; aircraft). */
struct VehTrig {
    float sh, ch, ta, sg, cg;
};

template <int KIND>
__device__ __forceinline__ void veh_trig(const float x[7], VehTrig& T) {
    sincosf(x[4], &T.sh, &T.ch);
    T.ta = tanf(x[5]);
    if (KIND == KIND_WING) sincosf(x[6], &T.sg, &T.cg);
}

/* sin and cos of a0 + d from those of a0, for a stage's small angle offset
 * d: the angle-sum formulas with sin d and cos d from their Taylor series
 * (through d^7 and d^8: remainders below 6e-11 for |d| <= 0.3, past FP32
 * rounding);
 * larger offsets (very long time steps) call sincosf. */
__device__ __forceinline__ void sincos_shift(float a0, float s0, float c0, float d, float& s, float& c) {
#pragma clang fp contract(off)
    if (fabsf(d) <= 0.3f) {
        const float d2 = d * d;
        const float sd = d * POTATO_FMA(-d2 * (1.0f / 6.0f), POTATO_FMA(-d2, 1.0f / 20.0f * POTATO_FMA(-d2, 1.0f / 42.0f, 1.0f), 1.0f), 1.0f);
        const float cm = d2 * 0.5f * POTATO_FMA(-d2, 1.0f / 12.0f * POTATO_FMA(-d2, 1.0f / 30.0f * POTATO_FMA(-d2, 1.0f / 56.0f, 1.0f), 1.0f), 1.0f);
        /* cos d = 1 - cm */
        s = POTATO_FMA(c0, sd, POTATO_FMA(-s0, cm, s0));
        c = POTATO_FMA(-s0, sd, POTATO_FMA(-c0, cm, c0));
    } else {
        sincosf(a0 + d, &s, &c);
    }
}

/* tan(a0 + d) from t0 = tan(a0): (t0 + tan d) / (1 - t0 tan d), tan d from
 * its series through d^7 (the remainder is below 3e-10 of tan d for
 * |d| <= 0.1); larger offsets, or a denominator that would cancel, call
 * tanf. */
__device__ __forceinline__ float tan_shift(float a0, float t0, float d) {
#pragma clang fp contract(off)
    const float d2 = d * d;
    const float td = d * POTATO_FMA(d2 * (1.0f / 3.0f), POTATO_FMA(d2, 0.4f * POTATO_FMA(d2, 17.0f / 42.0f, 1.0f), 1.0f), 1.0f);
    const float den = POTATO_FMA(-t0, td, 1.0f);
    if (fabsf(d) <= 0.1f && den >= 0.5f) return (t0 + td) / den;
    return tanf(a0 + d);
}

/* The angles' functions at a stage state x0 + offsets (h k of the previous
 * stage's rates) from those at x0. */
template <int KIND>
__device__ __forceinline__ void veh_trig_shift(const float x0[7], const VehTrig& T0, float h, const float k[7],
                                               VehTrig& T) {
    sincos_shift(x0[4], T0.sh, T0.ch, h * k[4], T.sh, T.ch);
    T.ta = tan_shift(x0[5], T0.ta, h * k[5]);
    if (KIND == KIND_WING) sincos_shift(x0[6], T0.sg, T0.cg, h * k[6], T.sg, T.cg);
}

/* Rates of rows 0-6 at state x (its angles' functions in T) with inputs u
 * held. */
template <int KIND>
__device__ __forceinline__ void veh_rates(const VehConst& c, const float x[7], const VehTrig& T, const float u[3],
                                          float dx[7]) {
#pragma clang fp contract(off)
    if (KIND == KIND_CAR) {
        const float td = T.ta;
        const float tb = c.lr_L * td;                         /* tan(beta) */
        const float cb = rsq(POTATO_FMA(tb, tb, 1.0f));       /* cos(beta) > 0 */
        const float sb = tb * cb;                             /* sin(beta) */
        const float cc = POTATO_FMA(T.ch, cb, -(T.sh * sb));  /* cos(psi + beta) */
        const float sc = POTATO_FMA(T.sh, cb, T.ch * sb);     /* sin(psi + beta) */
        dx[0] = x[3] * cc;
        dx[1] = x[3] * sc;
        dx[2] = 0.0f;
        dx[3] = POTATO_FMA(-c.cd_m, x[3], u[0]);
        dx[4] = (x[3] * cb) * (td * c.inv_L);
        dx[5] = (u[1] - x[5]) * c.inv_tau[0];
        dx[6] = 0.0f;
    } else {
        const float vh = x[3] * T.cg;                         /* horizontal speed */
        dx[0] = vh * T.ch;
        dx[1] = vh * T.sh;
        dx[2] = x[3] * T.sg;
        dx[3] = (u[0] - x[3]) * c.inv_tau[0];
        dx[4] = (c.g * T.ta) / x[3];
        dx[5] = (u[1] - x[5]) * c.inv_tau[1];
        dx[6] = (u[2] - x[6]) * c.inv_tau[2];
    }
}

/* Closed-loop inputs from the step-start state x (its angles' functions in
 * T) around orbit centre wp. */
template <int KIND>
__device__ __forceinline__ void veh_guidance(const VehConst& c, const float x[7], const VehTrig& T, const float wp[3],
                                             float u[3]) {
#pragma clang fp contract(off)
    const float ex = x[0] - wp[0], ey = x[1] - wp[1];
    const float d = sqrtf(POTATO_FMA(ey, ey, ex * ex));
    const float chi_d = POTATO_FMA(c.lam, atanf(c.k_orb_rho * (d - c.rho)), atan2f(ey, ex) + c.lam_half_pi);
    if (KIND == KIND_CAR) {
        /* the car's course is its yaw plus the side-slip angle */
        const float beta = atanf(c.lr_L * T.ta);
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

/* Classical RK4 over rows 0-6 with the inputs held, from the step-start
 * state x whose angles' functions are T; CARRY: every integrated row keeps
 * its rounding carry in lo (the heading matters most: it grows by nearly
 * equal increments every step, and a rounding bias of its updates would be
 * cancelled by a steady steering or bank offset). */
template <int KIND, bool CARRY>
__device__ __forceinline__ void veh_rk4(const VehConst& c, const Limits& L, float x[7], const VehTrig& T, float lo[7],
                                        const float u[3]) {
#pragma clang fp contract(off)
    float k[7], acc[7], xs[7];
    VehTrig Ts;
    veh_rates<KIND>(c, x, T, u, k);
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        acc[i] = k[i];
        xs[i] = veh_row<KIND>(i) ? POTATO_FMA(L.half_dt, k[i], x[i]) : x[i];
    }
    veh_trig_shift<KIND>(x, T, L.half_dt, k, Ts);
    veh_rates<KIND>(c, xs, Ts, u, k);
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        acc[i] = POTATO_FMA(2.0f, k[i], acc[i]);
        xs[i] = veh_row<KIND>(i) ? POTATO_FMA(L.half_dt, k[i], x[i]) : x[i];
    }
    veh_trig_shift<KIND>(x, T, L.half_dt, k, Ts);
    veh_rates<KIND>(c, xs, Ts, u, k);
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        acc[i] = POTATO_FMA(2.0f, k[i], acc[i]);
        xs[i] = veh_row<KIND>(i) ? POTATO_FMA(L.dt, k[i], x[i]) : x[i];
    }
    veh_trig_shift<KIND>(x, T, L.dt, k, Ts);
    veh_rates<KIND>(c, xs, Ts, u, k);
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        if (!veh_row<KIND>(i)) continue;
        add_carry<CARRY>(x[i], lo[i], L.dt6 * (acc[i] + k[i]));
    }
}

}  // namespace potato
