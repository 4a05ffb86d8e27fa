/*
 * quad_step.h -- per-agent FP32 arithmetic of one quadrotor time step, for
 * gfx950 kernels (one agent per lane, everything in registers).
 *
 * The physics follows Sec. II-B of the paper: eqs. (qd1)-(qd4) for the rigid
 * body, eq. (2) for rotor thrust/torque, eq. (3) for the allocation matrix,
 * classical RK4 for the discretisation, and a PID cascade ending in the
 * body-rate loop.  Differences from a literal transcription, all exact
 * algebraic rewrites chosen for FP32 accuracy or speed:
 *   - rotor speeds are carried as d = W - w_ref, and squared speeds as
 *     s = W^2 - w_ref^2 = d (2 w_ref + d), so the small speed differences
 *     that make the torques are not lost against a large W;
 *   - collective thrust over mass is F0 + (k_f/m) sum(s), F0 = 4 k_f w_ref^2 / m,
 *     and the vertical acceleration is assembled as (F0 - g) + ... so that
 *     the hover cancellation thrust/m - g happens once, on the host;
 *   - the mixer uses the closed-form inverse G^-1 = G^T diag(1/|row|^2),
 *     exact because the rows of G are mutually orthogonal;
 *   - divisions by mass, inertia, tau_m and dt are multiplications by
 *     reciprocals precomputed per type.
 * The reference FP64 implementation performs the literal operations; the
 * two agree to the tolerance the tests state.
 */
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace potato {

/* Per-type constants, derived once on the host from potato_type_params and
 * rounded to FP32. */
struct TypeConst {
    float mass, inv_m, cd_m;              /* m, 1/m, c_d/m */
    float Ix, Iy, Iz, iIx, iIy, iIz;      /* inertia and its inverse */
    float F0, F0_g, kf_m;                 /* 4 k_f w_ref^2/m, F0 - g, k_f/m */
    float kf_ls, kf_lc, km;               /* k_f L sin(a), k_f L cos(a), k_m */
    float w_ref, two_w, four_w2;          /* w_ref, 2 w_ref, 4 w_ref^2 */
    float inv_tau;                        /* 1 / tau_m */
    float mix_x, mix_y, mix_z;            /* 1/(4 L sin a), 1/(4 L cos a), k_f/(4 k_m) */
    float f_max, inv_kf;                  /* k_f w_max^2, 1/k_f */
    float gains[9];
    int32_t budget;
    int32_t pad_;
};

/* Controller limits and the time step, shared by all agents of a launch. */
struct Limits {
    float g, r_sat, r_sat2, ipos_max, iatt_max, irate_max, az_min;
    float dt, half_dt, dt6, inv_dt;
};

struct Gains {
    float kpp, kip, kdp, kpa, kia, kda, kpr, kir, kdr;
};

/* 17 integrated rows + running cost, plus the controller memory. */
struct Agent {
    float p[3], v[3], q[4], w[3], d[4];   /* d = rotor speed - w_ref */
    float J;
    float ip[3], ia[3], ir[3], wprev[3];
    float p_lo[3], v_lo[3], J_lo;         /* rounding carries of p, v, J */
};

/* x += inc with the rounding error carried in lo (Fast2Sum, Dekker 1971):
 * the carried low part is added back into the next increment, so a long
 * run of nearly equal increments does not drift by half an ulp per step. */
__device__ __forceinline__ void add_carry(float& x, float& lo, float inc) {
    const float y = inc + lo;
    const float s = x + y;
    lo = y - (s - x);
    x = s;
}

__device__ __forceinline__ float clampf_(float x, float lo, float hi) {
    return x < lo ? lo : (x > hi ? hi : x);
}

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float sqrt_fast(float x) { return __builtin_amdgcn_sqrtf(x); }

/* Body z axis in the inertial frame: third column of R(q), unit-norm form
 * (eq. qd2 with thrust along body z). */
__device__ __forceinline__ void body_z(const float q[4], float bz[3]) {
    bz[0] = 2.0f * (q[1] * q[3] + q[0] * q[2]);
    bz[1] = 2.0f * (q[2] * q[3] - q[0] * q[1]);
    bz[2] = 1.0f - 2.0f * (q[1] * q[1] + q[2] * q[2]);
}

/* Rate of the integrated rows for held rotor command dc (relative to w_ref).
 * Position is not an input: only its derivative (= v) is needed.  Outputs
 * dv, dq, dw, dd and the cost rate dJ. */
__device__ __forceinline__ void derivative(const TypeConst& c, const float v[3], const float q[4],
                                           const float w[3], const float d[4], const float dc[4],
                                           float dv[3], float dq[4], float dw[3], float dd[4],
                                           float& dJ) {
    /* eq. (2) with s_i = W_i^2 - w_ref^2 */
    float s[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) s[i] = d[i] * (c.two_w + d[i]);
    const float ssum = (s[0] + s[1]) + (s[2] + s[3]);
    /* eq. (3): body torques from the rotor thrusts */
    const float tx = c.kf_ls * ((s[0] - s[1]) + (s[3] - s[2]));
    const float ty = c.kf_lc * ((s[2] - s[0]) + (s[3] - s[1]));
    const float tz = c.km * ((s[0] - s[1]) + (s[2] - s[3]));
    /* eq. (qd2) + drag: (f_c/m) R(q) z - (c_d/m) v - g z */
    const float ftm = c.F0 + c.kf_m * ssum;
    const float x2y2 = q[1] * q[1] + q[2] * q[2];
    const float bx = 2.0f * (q[1] * q[3] + q[0] * q[2]);
    const float by = 2.0f * (q[2] * q[3] - q[0] * q[1]);
    dv[0] = ftm * bx - c.cd_m * v[0];
    dv[1] = ftm * by - c.cd_m * v[1];
    dv[2] = (c.F0_g + c.kf_m * ssum) - 2.0f * ftm * x2y2 - c.cd_m * v[2];
    /* eq. (qd3): q' = 1/2 q o (0, w) */
    dq[0] = -0.5f * (q[1] * w[0] + q[2] * w[1] + q[3] * w[2]);
    dq[1] = 0.5f * (q[0] * w[0] + q[2] * w[2] - q[3] * w[1]);
    dq[2] = 0.5f * (q[0] * w[1] + q[3] * w[0] - q[1] * w[2]);
    dq[3] = 0.5f * (q[0] * w[2] + q[1] * w[1] - q[2] * w[0]);
    /* eq. (qd4): w' = I^-1 (tau - w x I w) */
    const float Iwx = c.Ix * w[0], Iwy = c.Iy * w[1], Iwz = c.Iz * w[2];
    dw[0] = c.iIx * (tx - (w[1] * Iwz - w[2] * Iwy));
    dw[1] = c.iIy * (ty - (w[2] * Iwx - w[0] * Iwz));
    dw[2] = c.iIz * (tz - (w[0] * Iwy - w[1] * Iwx));
    /* first-order rotor lag */
#pragma unroll
    for (int i = 0; i < 4; ++i) dd[i] = (dc[i] - d[i]) * c.inv_tau;
    dJ = c.four_w2 + ssum;
}

/* Position -> attitude -> body-rate PID cascade and mixer, evaluated once
 * per step on the step-start state; returns rotor commands relative to
 * w_ref and updates the controller memory. */
__device__ __forceinline__ void controller(const TypeConst& c, const Limits& L, const Gains& k,
                                           Agent& a, const float wp[3], float dc[4]) {
    /* position loop: error saturated to radius r_sat */
    float e[3] = {wp[0] - a.p[0], wp[1] - a.p[1], wp[2] - a.p[2]};
    const float n2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
    if (n2 > L.r_sat2) {
        const float sc = L.r_sat * rsq(n2);
        e[0] *= sc; e[1] *= sc; e[2] *= sc;
    }
    float acc[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        a.ip[i] = clampf_(a.ip[i] + e[i] * L.dt, -L.ipos_max, L.ipos_max);
        acc[i] = k.kpp * e[i] + k.kip * a.ip[i] - k.kdp * a.v[i];
    }
    acc[2] += L.g;
    acc[2] = acc[2] < L.az_min ? L.az_min : acc[2];

    /* collective thrust: commanded acceleration along the current body z */
    float bz[3];
    body_z(a.q, bz);
    const float fc = c.mass * (acc[0] * bz[0] + acc[1] * bz[1] + acc[2] * bz[2]);

    /* desired attitude: shortest rotation of z onto the thrust direction */
    const float ra = rsq(acc[0] * acc[0] + acc[1] * acc[1] + acc[2] * acc[2]);
    const float nx = acc[0] * ra, ny = acc[1] * ra, nz = acc[2] * ra;
    float qd0 = 1.0f + nz, qd1 = -ny, qd2 = nx;
    const float rq = rsq(qd0 * qd0 + qd1 * qd1 + qd2 * qd2);
    qd0 *= rq; qd1 *= rq; qd2 *= rq;

    /* attitude loop on conj(q) o q_des (short arc) */
    const float* q = a.q;
    float ew = q[0] * qd0 + q[1] * qd1 + q[2] * qd2;
    float ex = q[0] * qd1 - q[1] * qd0 + q[3] * qd2;
    float ey = q[0] * qd2 - q[2] * qd0 - q[3] * qd1;
    float ez = q[2] * qd1 - q[1] * qd2 - q[3] * qd0;
    const float sg = ew < 0.0f ? -2.0f : 2.0f;
    const float eatt[3] = {sg * ex, sg * ey, sg * ez};
    float alpha[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        a.ia[i] = clampf_(a.ia[i] + eatt[i] * L.dt, -L.iatt_max, L.iatt_max);
        const float wdes = k.kpa * eatt[i] + k.kia * a.ia[i] - k.kda * a.w[i];
        /* body-rate loop, derivative on the measured rate */
        const float erate = wdes - a.w[i];
        a.ir[i] = clampf_(a.ir[i] + erate * L.dt, -L.irate_max, L.irate_max);
        alpha[i] = k.kpr * erate + k.kir * a.ir[i] - k.kdr * ((a.w[i] - a.wprev[i]) * L.inv_dt);
        a.wprev[i] = a.w[i];
    }
    /* torque for the desired angular acceleration, eq. (qd4) inverted */
    const float Iwx = c.Ix * a.w[0], Iwy = c.Iy * a.w[1], Iwz = c.Iz * a.w[2];
    const float tx = c.Ix * alpha[0] + (a.w[1] * Iwz - a.w[2] * Iwy);
    const float ty = c.Iy * alpha[1] + (a.w[2] * Iwx - a.w[0] * Iwz);
    const float tz = c.Iz * alpha[2] + (a.w[0] * Iwy - a.w[1] * Iwx);

    /* mixer: f = G^-1 [fc, tau], saturate, invert eq. (2) */
    const float f4 = 0.25f * fc;
    const float X = tx * c.mix_x, Y = ty * c.mix_y, Z = tz * c.mix_z;
    float f[4];
    f[0] = f4 + X - Y + Z;
    f[1] = f4 - X - Y - Z;
    f[2] = f4 - X + Y + Z;
    f[3] = f4 + X + Y - Z;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float fi = clampf_(f[i], 0.0f, c.f_max);
        dc[i] = sqrt_fast(fi * c.inv_kf) - c.w_ref;
    }
}

/* Classical RK4 with the command held, then quaternion renormalisation. */
__device__ __forceinline__ void rk4_step(const TypeConst& c, const Limits& L, Agent& a,
                                         const float dc[4]) {
    float sv[3], sq[4], sw[3], sd[4];      /* stage state */
    float kv[3], kq[4], kw[3], kd[4], kJ;  /* stage rate */
    float av[3], aq[4], aw[3], ad[4], ap[3], aJ;  /* weighted sum of rates */

    derivative(c, a.v, a.q, a.w, a.d, dc, kv, kq, kw, kd, kJ);
#pragma unroll
    for (int i = 0; i < 3; ++i) { ap[i] = a.v[i]; av[i] = kv[i]; aw[i] = kw[i]; }
#pragma unroll
    for (int i = 0; i < 4; ++i) { aq[i] = kq[i]; ad[i] = kd[i]; }
    aJ = kJ;
#pragma unroll
    for (int i = 0; i < 3; ++i) { sv[i] = a.v[i] + L.half_dt * kv[i]; sw[i] = a.w[i] + L.half_dt * kw[i]; }
#pragma unroll
    for (int i = 0; i < 4; ++i) { sq[i] = a.q[i] + L.half_dt * kq[i]; sd[i] = a.d[i] + L.half_dt * kd[i]; }

    derivative(c, sv, sq, sw, sd, dc, kv, kq, kw, kd, kJ);
#pragma unroll
    for (int i = 0; i < 3; ++i) { ap[i] += 2.0f * sv[i]; av[i] += 2.0f * kv[i]; aw[i] += 2.0f * kw[i]; }
#pragma unroll
    for (int i = 0; i < 4; ++i) { aq[i] += 2.0f * kq[i]; ad[i] += 2.0f * kd[i]; }
    aJ += 2.0f * kJ;
#pragma unroll
    for (int i = 0; i < 3; ++i) { sv[i] = a.v[i] + L.half_dt * kv[i]; sw[i] = a.w[i] + L.half_dt * kw[i]; }
#pragma unroll
    for (int i = 0; i < 4; ++i) { sq[i] = a.q[i] + L.half_dt * kq[i]; sd[i] = a.d[i] + L.half_dt * kd[i]; }

    derivative(c, sv, sq, sw, sd, dc, kv, kq, kw, kd, kJ);
#pragma unroll
    for (int i = 0; i < 3; ++i) { ap[i] += 2.0f * sv[i]; av[i] += 2.0f * kv[i]; aw[i] += 2.0f * kw[i]; }
#pragma unroll
    for (int i = 0; i < 4; ++i) { aq[i] += 2.0f * kq[i]; ad[i] += 2.0f * kd[i]; }
    aJ += 2.0f * kJ;
#pragma unroll
    for (int i = 0; i < 3; ++i) { sv[i] = a.v[i] + L.dt * kv[i]; sw[i] = a.w[i] + L.dt * kw[i]; }
#pragma unroll
    for (int i = 0; i < 4; ++i) { sq[i] = a.q[i] + L.dt * kq[i]; sd[i] = a.d[i] + L.dt * kd[i]; }

    derivative(c, sv, sq, sw, sd, dc, kv, kq, kw, kd, kJ);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        ap[i] += sv[i]; av[i] += kv[i]; aw[i] += kw[i];
        add_carry(a.p[i], a.p_lo[i], L.dt6 * ap[i]);
        add_carry(a.v[i], a.v_lo[i], L.dt6 * av[i]);
        a.w[i] += L.dt6 * aw[i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        aq[i] += kq[i]; ad[i] += kd[i];
        a.q[i] += L.dt6 * aq[i];
        a.d[i] += L.dt6 * ad[i];
    }
    aJ += kJ;
    add_carry(a.J, a.J_lo, L.dt6 * aJ);

    const float r = rsq(a.q[0] * a.q[0] + a.q[1] * a.q[1] + a.q[2] * a.q[2] + a.q[3] * a.q[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i) a.q[i] *= r;
}

}  // namespace potato
