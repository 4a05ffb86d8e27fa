/*
 * quad_adjoint.h -- hand-written reverse mode (vector-Jacobian product) of
 * one quadrotor time step, FP32, one agent per lane.
 *
 * Forward step (quad_step.h): controller -> held rotor command dc; classical
 * RK4 over v, q, w, d (and p, J, which only integrate) with dc held;
 * quaternion renormalisation.  step_vjp() recomputes the forward
 * intermediates of one step from its step-start state and then applies the
 * transposed derivatives in reverse order:
 *     renormalisation -> RK4 stages 4, 3, 2, 1 -> controller.
 * Non-smooth points take the derivative of the branch the forward pass
 * took: a clamp passes the cotangent inside its interval and stops it
 * outside; the error-quaternion sign is a constant; sqrt'(0) is taken as 0.
 * The branches are the forward's own decisions, recorded on the tape by the
 * recomputation (which replays the forward bit for bit), as is the rotor
 * command it held through the step; the reverse sweep does not decide any
 * branch itself.  The rounding carries of the forward integrator are not
 * differentiated (the represented value is row + carry, so both have the
 * same cotangent).
 */
#pragma once

#include "kernels.h"
#include "quad_step.h"

namespace potato {

/* Cotangents of the 30 physical state rows. */
struct AgentAdj {
    float p[3], v[3], q[4], w[3], d[4], J;
    float ip[3], ia[3], ir[3], wprev[3];
};

/* Cotangent of the integrated rates of (v, q, w, d, J); the position rate
 * is v itself and is folded in by the caller.  qh holds half the cotangent
 * of the quaternion rate q o (0, w) / 2, i.e. the cotangent of q o (0, w),
 * so the kinematics need no factor. */
struct RateAdj {
    float v[3], qh[4], w[3], d[4], J;
};

/* Dynamic part of the state seen by the right-hand side. */
struct Dyn {
    float v[3], q[4], w[3], d[4];
};

/* Transpose of the Jacobian of the right-hand side (eqs. qd2-qd4, 2, 3 and
 * the rotor lag) at y, applied to mu.  Adds the state cotangent to
 * (lv, lq, lw, ld); the rotor-command cotangent, inv_tau times the
 * rotor-rate cotangent, is formed by the caller from the summed mu.d.
 * Products with inverse inertia use the per-type constants of the forward
 * step: (I_z - I_y)/I_x = gx etc., k_f L sin(a)/I_x = ax etc. */
__device__ __forceinline__ void derivative_vjp(const TypeConst& c, const Dyn& y, const RateAdj& mu,
                                               float lv[3], float lq[4], float lw[3], float ld[4]) {
    const float* q = y.q;
    const float* w = y.w;
    float s[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) s[i] = y.d[i] * (c.two_w + y.d[i]);
    const float ssum = (s[0] + s[1]) + (s[2] + s[3]);
    const float ftm = c.F0 + c.kf_m * ssum;
    const float x2y2 = q[1] * q[1] + q[2] * q[2];
    const float hbx = q[1] * q[3] + q[0] * q[2];      /* half of R(q) z, x and y */
    const float hby = q[2] * q[3] - q[0] * q[1];

    /* translational part: v' = 2 ftm (hbx, hby, 1/2 - x2y2) - (c_d/m) v - g z */
    const float l_ftm = 2.0f * (mu.v[0] * hbx + mu.v[1] * hby - mu.v[2] * x2y2);
    const float l_ssum = c.kf_m * (l_ftm + mu.v[2]) + mu.J;
    const float m0 = 2.0f * ftm * mu.v[0], m1 = 2.0f * ftm * mu.v[1], m2 = 4.0f * ftm * mu.v[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) lv[i] -= c.cd_m * mu.v[i];
    lq[0] += m0 * q[2] - m1 * q[1];
    lq[1] += m0 * q[3] - m1 * q[0] - m2 * q[1];
    lq[2] += m0 * q[0] + m1 * q[3] - m2 * q[2];
    lq[3] += m0 * q[1] + m1 * q[2];

    /* quaternion kinematics q o (0, w), cotangent mu.qh */
    const float* m = mu.qh;
    lq[0] += w[0] * m[1] + w[1] * m[2] + w[2] * m[3];
    lq[1] += -w[0] * m[0] - w[2] * m[2] + w[1] * m[3];
    lq[2] += -w[1] * m[0] + w[2] * m[1] - w[0] * m[3];
    lq[3] += -w[2] * m[0] - w[1] * m[1] + w[0] * m[2];
    lw[0] += -q[1] * m[0] + q[0] * m[1] + q[3] * m[2] - q[2] * m[3];
    lw[1] += -q[2] * m[0] - q[3] * m[1] + q[0] * m[2] + q[1] * m[3];
    lw[2] += -q[3] * m[0] + q[2] * m[1] - q[1] * m[2] + q[0] * m[3];

    /* Euler's equations: w' = (ax (A + B), ay (P23 - P01), az (A - B)) - (gx w1 w2, gy w2 w0, gz w0 w1) */
    const float b0 = c.gx * mu.w[0], b1 = c.gy * mu.w[1], b2 = c.gz * mu.w[2];
    lw[0] -= b1 * w[2] + b2 * w[1];
    lw[1] -= b0 * w[2] + b2 * w[0];
    lw[2] -= b0 * w[1] + b1 * w[0];

    /* rotor model and allocation (eqs. 2, 3) through s_i = W_i^2 - w_ref^2 */
    const float tX = c.ax * mu.w[0], tY = c.ay * mu.w[1], tZ = c.az * mu.w[2];
    const float pz = l_ssum + tZ, mz = l_ssum - tZ, u = tX - tY, v = tX + tY;
    const float lsv[4] = {pz + u, mz - v, pz - u, mz + v};
#pragma unroll
    for (int i = 0; i < 4; ++i)
        ld[i] += lsv[i] * (c.two_w + 2.0f * y.d[i]) - c.inv_tau * mu.d[i];
}

/*
 * Reverse of one step.  `a` is the step-start state (as the forward pass
 * saw it; its J and carries are not read), wp the waypoint of this step, k
 * the gains, dc the rotor command the forward controller held through the
 * step and bits its branch decisions (kBit*).  lam holds the cotangent of
 * the step-end state on entry and of the step-start state on return; gk
 * accumulates the gain cotangents.
 */
__device__ __forceinline__ void step_vjp(const TypeConst& c, const Limits& L, const Gains& k,
                                         const Agent& a, const float wp[3], const float dc[4],
                                         uint32_t bits, AgentAdj& lam, float gk[9]) {
    /* ---------------- RK4 forward, keeping the stage states ----------------
     * (the forward step's own arithmetic: rates() with the quaternion rate's
     * factor 1/2 on the step sizes, and the rotor lag's closed-form stage
     * values, so the stage states are the forward's bits) */
    const float z = -(L.dt * c.inv_tau);
    const float hz = 0.5f * z;
    const float c2 = 1.0f + hz;
    const float c3 = __builtin_fmaf(hz, c2, 1.0f);
    const float c4 = __builtin_fmaf(z, c3, 1.0f);
    float e_d[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) e_d[i] = a.d[i] - dc[i];
    Dyn y1, y2, y3, y4;
    float kv[3], kq[4], kw[3], aq[4];
#pragma unroll
    for (int i = 0; i < 3; ++i) { y1.v[i] = a.v[i]; y1.w[i] = a.w[i]; }
#pragma unroll
    for (int i = 0; i < 4; ++i) { y1.q[i] = a.q[i]; y1.d[i] = a.d[i]; }
    auto stage = [&](const Dyn& from, float hvw, float hq, float cp, Dyn& to) {
        rates(c, from.v, from.q, from.w, from.d, kv, kq, kw);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            to.v[i] = __builtin_fmaf(hvw, kv[i], y1.v[i]);
            to.w[i] = __builtin_fmaf(hvw, kw[i], y1.w[i]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            to.q[i] = __builtin_fmaf(hq, kq[i], y1.q[i]);
            to.d[i] = __builtin_fmaf(e_d[i], cp, dc[i]);
        }
    };
    stage(y1, L.half_dt, L.quarter_dt, c2, y2);
#pragma unroll
    for (int i = 0; i < 4; ++i) aq[i] = kq[i];
    stage(y2, L.half_dt, L.quarter_dt, c3, y3);
#pragma unroll
    for (int i = 0; i < 4; ++i) aq[i] = __builtin_fmaf(2.0f, kq[i], aq[i]);
    stage(y3, L.dt, L.half_dt, c4, y4);
#pragma unroll
    for (int i = 0; i < 4; ++i) aq[i] = __builtin_fmaf(2.0f, kq[i], aq[i]);
    rates(c, y4.v, y4.q, y4.w, y4.d, kv, kq, kw);
    float qn[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) qn[i] = __builtin_fmaf(L.dt12, aq[i] + kq[i], a.q[i]);

    /* ---------------- reverse: renormalisation ---------------- */
    {
        const float r = rsq(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
        const float u[4] = {qn[0] * r, qn[1] * r, qn[2] * r, qn[3] * r};
        const float dot = u[0] * lam.q[0] + u[1] * lam.q[1] + u[2] * lam.q[2] + u[3] * lam.q[3];
#pragma unroll
        for (int i = 0; i < 4; ++i) lam.q[i] = r * (lam.q[i] - u[i] * dot);
    }

    /* ---------------- reverse: RK4 ----------------
     * lam (v, q, w, d) is the cotangent of the step-end dynamic state; the
     * stage rate cotangents are b_i * dt * lam + dt * (cotangent of the next
     * stage state), with b = 1/6, 1/3, 1/3, 1/6.  Position and cost only
     * integrate, so their cotangents pass through unchanged and enter each
     * stage as b_i * dt * lam.p (on the stage velocity) and b_i * dt * lam.J. */
    const AgentAdj lo = lam;                 /* cotangent of the step end */
    float mdsum[4] = {0.0f, 0.0f, 0.0f, 0.0f};   /* rotor-rate cotangents summed over the stages */
    float sv[3], sq[4], sw[3], sd[4];        /* running stage-state cotangent */
    const float bw[4] = {L.dt6, 2.0f * L.dt6, 2.0f * L.dt6, L.dt6};
    const float hs[4] = {0.0f, L.half_dt, L.half_dt, L.dt};   /* stage offsets */
    /* the same halved, for the quaternion-rate cotangent mu.qh */
    const float bwh[4] = {L.dt12, L.dt6, L.dt6, L.dt12};
    const float hsh[4] = {0.0f, L.quarter_dt, L.quarter_dt, L.half_dt};
#pragma unroll
    for (int i = 0; i < 3; ++i) { sv[i] = 0.0f; sw[i] = 0.0f; }
#pragma unroll
    for (int i = 0; i < 4; ++i) { sq[i] = 0.0f; sd[i] = 0.0f; }
#pragma unroll
    for (int st = 3; st >= 0; --st) {
        /* cotangent of this stage's rate: b dt lam_end + h_{next} lam_{next stage} */
        const float hn = st < 3 ? hs[st + 1] : 0.0f;
        const float hnh = st < 3 ? hsh[st + 1] : 0.0f;
        RateAdj mu;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            mu.v[i] = bw[st] * lo.v[i] + hn * sv[i];
            mu.w[i] = bw[st] * lo.w[i] + hn * sw[i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            mu.qh[i] = bwh[st] * lo.q[i] + hnh * sq[i];
            mu.d[i] = bw[st] * lo.d[i] + hn * sd[i];
            mdsum[i] += mu.d[i];
        }
        mu.J = bw[st] * lo.J;
        const Dyn& ys = st == 3 ? y4 : (st == 2 ? y3 : (st == 1 ? y2 : y1));
        float nv_[3], nq_[4], nw_[3], nd_[4];
        /* position rate is the stage velocity */
#pragma unroll
        for (int i = 0; i < 3; ++i) { nv_[i] = bw[st] * lo.p[i]; nw_[i] = 0.0f; }
#pragma unroll
        for (int i = 0; i < 4; ++i) { nq_[i] = 0.0f; nd_[i] = 0.0f; }
        derivative_vjp(c, ys, mu, nv_, nq_, nw_, nd_);
        /* stage state = y1 + h_st * previous rate: cotangent flows to y1 and
         * (scaled by h_st) to the previous stage's rate */
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            sv[i] = nv_[i]; sw[i] = nw_[i];
            lam.v[i] += nv_[i]; lam.w[i] += nw_[i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            sq[i] = nq_[i]; sd[i] = nd_[i];
            lam.q[i] += nq_[i]; lam.d[i] += nd_[i];
        }
    }
    float ldc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) ldc[i] = c.inv_tau * mdsum[i];

    /* ---------------- controller, forward with intermediates ----------------
     * (the values the reverse needs; the branches are the recorded ones) */
    float er[3] = {wp[0] - a.p[0], wp[1] - a.p[1], wp[2] - a.p[2]};
    const float n2 = er[0] * er[0] + er[1] * er[1] + er[2] * er[2];
    const bool sat = (bits & kBitSat) != 0;
    float rs = 0.0f, sc = 1.0f;
    if (sat) { rs = rsq(n2); sc = L.r_sat * rs; }
    const float e[3] = {er[0] * sc, er[1] * sc, er[2] * sc};
    float ipn[3];
    bool in_ip[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float pre = a.ip[i] + e[i] * L.dt;
        in_ip[i] = (bits & (kBitIp << i)) != 0;
        ipn[i] = clampf_(pre, -L.ipos_max, L.ipos_max);
    }
    float acc[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) acc[i] = k.kpp * e[i] + k.kip * ipn[i] - k.kdp * a.v[i];
    acc[2] += L.g;
    const bool az_cl = (bits & kBitAz) != 0;
    if (az_cl) acc[2] = L.az_min;
    float bz[3];
    body_z(a.q, bz);
    const float ra = rsq(acc[0] * acc[0] + acc[1] * acc[1] + acc[2] * acc[2]);
    const float nv[3] = {acc[0] * ra, acc[1] * ra, acc[2] * ra};
    const float qr0 = 1.0f + nv[2], qr1 = -nv[1], qr2 = nv[0];
    const float rq = rsq(qr0 * qr0 + qr1 * qr1 + qr2 * qr2);
    const float qd[3] = {qr0 * rq, qr1 * rq, qr2 * rq};
    const float* q = a.q;
    const float qex = q[0] * qd[1] - q[1] * qd[0] + q[3] * qd[2];
    const float qey = q[0] * qd[2] - q[2] * qd[0] - q[3] * qd[1];
    const float qez = q[2] * qd[1] - q[1] * qd[2] - q[3] * qd[0];
    const float sg = (bits & kBitSgn) != 0 ? -2.0f : 2.0f;
    const float eatt[3] = {sg * qex, sg * qey, sg * qez};
    float ian[3], irn[3], wdes[3], erate[3];
    bool in_ia[3], in_ir[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float pa = a.ia[i] + eatt[i] * L.dt;
        in_ia[i] = (bits & (kBitIa << i)) != 0;
        ian[i] = clampf_(pa, -L.iatt_max, L.iatt_max);
        wdes[i] = k.kpa * eatt[i] + k.kia * ian[i] - k.kda * a.w[i];
        erate[i] = wdes[i] - a.w[i];
        const float pr = a.ir[i] + erate[i] * L.dt;
        in_ir[i] = (bits & (kBitIr << i)) != 0;
        irn[i] = clampf_(pr, -L.irate_max, L.irate_max);
    }
    /* rotor speed W = sqrt(f / k_f) of the held command: dW/df = 1 / (2 k_f W),
     * zero where the thrust was clamped or W == 0 */
    float lf_scale[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float W = dc[i] + c.w_ref;
        lf_scale[i] = (bits & (kBitRotor << i)) != 0 ? 0.5f * c.inv_kf * __builtin_amdgcn_rcpf(W) : 0.0f;
    }

    /* ---------------- reverse: controller ---------------- */
    float lf[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) lf[i] = ldc[i] * lf_scale[i];
    const float l_f4 = lf[0] + lf[1] + lf[2] + lf[3];
    const float l_X = lf[0] - lf[1] - lf[2] + lf[3];
    const float l_Y = -lf[0] - lf[1] + lf[2] + lf[3];
    const float l_Z = lf[0] - lf[1] + lf[2] - lf[3];
    const float l_fc = 0.25f * l_f4;
    const float ltx = c.mix_x * l_X, lty = c.mix_y * l_Y, ltz = c.mix_z * l_Z;
    const float lal[3] = {c.Ix * ltx, c.Iy * lty, c.Iz * ltz};
    /* gyroscopic feed-forward w x (I w) */
    {
        const float gzy = c.Iz - c.Iy, gxz = c.Ix - c.Iz, gyx = c.Iy - c.Ix;
        lam.w[0] += lty * gxz * a.w[2] + ltz * gyx * a.w[1];
        lam.w[1] += ltx * gzy * a.w[2] + ltz * gyx * a.w[0];
        lam.w[2] += ltx * gzy * a.w[1] + lty * gxz * a.w[0];
    }
    float l_eatt[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        /* w_prev <- w */
        lam.w[i] += lo.wprev[i];
        /* rate loop */
        const float dwd = (a.w[i] - a.wprev[i]) * L.inv_dt;
        gk[6] += lal[i] * erate[i];
        gk[7] += lal[i] * irn[i];
        gk[8] -= lal[i] * dwd;
        float l_er = k.kpr * lal[i];
        const float l_irn = lo.ir[i] + k.kir * lal[i];
        lam.w[i] -= k.kdr * L.inv_dt * lal[i];
        lam.wprev[i] = k.kdr * L.inv_dt * lal[i];
        const float l_irpre = in_ir[i] ? l_irn : 0.0f;
        lam.ir[i] = l_irpre;
        l_er += L.dt * l_irpre;
        /* erate = wdes - w */
        const float l_wd = l_er;
        lam.w[i] -= l_er;
        /* attitude loop */
        gk[3] += l_wd * eatt[i];
        gk[4] += l_wd * ian[i];
        gk[5] -= l_wd * a.w[i];
        const float l_ian = lo.ia[i] + k.kia * l_wd;
        lam.w[i] -= k.kda * l_wd;
        const float l_iapre = in_ia[i] ? l_ian : 0.0f;
        lam.ia[i] = l_iapre;
        l_eatt[i] = k.kpa * l_wd + L.dt * l_iapre;
    }
    /* error quaternion (the sign is a constant of the branch) */
    const float lex = sg * l_eatt[0], ley = sg * l_eatt[1], lez = sg * l_eatt[2];
    lam.q[0] += lex * qd[1] + ley * qd[2];
    lam.q[1] += -lex * qd[0] - lez * qd[2];
    lam.q[2] += -ley * qd[0] + lez * qd[1];
    lam.q[3] += lex * qd[2] - ley * qd[1] - lez * qd[0];
    const float lqd[3] = {-lex * q[1] - ley * q[2] - lez * q[3],
                          lex * q[0] - ley * q[3] + lez * q[2],
                          lex * q[3] + ley * q[0] - lez * q[1]};
    /* normalisation of the desired-attitude quaternion */
    const float dqd = qd[0] * lqd[0] + qd[1] * lqd[1] + qd[2] * lqd[2];
    const float lqr0 = rq * (lqd[0] - qd[0] * dqd);
    const float lqr1 = rq * (lqd[1] - qd[1] * dqd);
    const float lqr2 = rq * (lqd[2] - qd[2] * dqd);
    /* q_raw = (1 + n_z, -n_y, n_x, 0) */
    const float ln[3] = {lqr2, -lqr1, lqr0};
    const float dn = nv[0] * ln[0] + nv[1] * ln[1] + nv[2] * ln[2];
    float la[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) la[i] = ra * (ln[i] - nv[i] * dn) + c.mass * l_fc * bz[i];
    /* body z axis used for the collective thrust */
    {
        const float m0 = c.mass * l_fc;
        const float lb0 = m0 * acc[0], lb1 = m0 * acc[1], lb2 = m0 * acc[2];
        lam.q[0] += 2.0f * (q[2] * lb0 - q[1] * lb1);
        lam.q[1] += 2.0f * (q[3] * lb0 - q[0] * lb1) - 4.0f * q[1] * lb2;
        lam.q[2] += 2.0f * (q[0] * lb0 + q[3] * lb1) - 4.0f * q[2] * lb2;
        lam.q[3] += 2.0f * (q[1] * lb0 + q[2] * lb1);
    }
    if (az_cl) la[2] = 0.0f;
    /* position loop */
    float l_e[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        gk[0] += la[i] * e[i];
        gk[1] += la[i] * ipn[i];
        gk[2] -= la[i] * a.v[i];
        lam.v[i] -= k.kdp * la[i];
        const float l_ipn = lo.ip[i] + k.kip * la[i];
        const float l_ippre = in_ip[i] ? l_ipn : 0.0f;
        lam.ip[i] = l_ippre;
        l_e[i] = k.kpp * la[i] + L.dt * l_ippre;
    }
    /* saturation e = r_sat * er / |er| */
    if (sat) {
        const float u[3] = {er[0] * rs, er[1] * rs, er[2] * rs};
        const float du = u[0] * l_e[0] + u[1] * l_e[1] + u[2] * l_e[2];
#pragma unroll
        for (int i = 0; i < 3; ++i) l_e[i] = sc * (l_e[i] - u[i] * du);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) lam.p[i] -= l_e[i];
}

/* Row accessors: `base` is row 0 of a [rows][ld] buffer, the same address
 * in every active lane, and `bo` the lane's byte offset (column index
 * times 4). */
template <typename T>
__device__ __forceinline__ T* row_ptr(T* base, int64_t ld, int k) {
    return uniform(base + k * ld);
}

__device__ __forceinline__ void load_rows(const float* base, int64_t ld, uint32_t bo, Agent& a, bool carries) {
    auto row = [&](int k) { return elem(row_ptr(base, ld, k), bo); };
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        a.p[k] = row(k); a.v[k] = row(3 + k); a.w[k] = row(10 + k);
        a.ip[k] = row(17 + k); a.ia[k] = row(20 + k);
        a.ir[k] = row(23 + k); a.wprev[k] = row(26 + k);
        a.p_lo[k] = carries ? row(30 + k) : 0.0f;
        a.v_lo[k] = carries ? row(33 + k) : 0.0f;
        a.ip_lo[k] = carries ? row(37 + k) : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) { a.q[k] = row(6 + k); a.d[k] = row(13 + k); }
    a.J = row(29);
    a.J_lo = carries ? row(36) : 0.0f;
}

__device__ __forceinline__ void load_adj(const float* base, int64_t ld, uint32_t bo, AgentAdj& l) {
    auto row = [&](int k) { return elem(row_ptr(base, ld, k), bo); };
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        l.p[k] = row(k); l.v[k] = row(3 + k); l.w[k] = row(10 + k);
        l.ip[k] = row(17 + k); l.ia[k] = row(20 + k);
        l.ir[k] = row(23 + k); l.wprev[k] = row(26 + k);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) { l.q[k] = row(6 + k); l.d[k] = row(13 + k); }
    l.J = row(29);
}

/* Cotangent of the initial state: rows 0-16 to x0 ([17][ld]), rows 17-29
 * to mem ([13][ld]) when it is given. */
__device__ __forceinline__ void store_adj(float* x0, float* mem, int64_t ld, uint32_t bo, const AgentAdj& l) {
    auto row = [&](int k) -> float& { return elem(row_ptr(x0, ld, k), bo); };
#pragma unroll
    for (int k = 0; k < 3; ++k) { row(k) = l.p[k]; row(3 + k) = l.v[k]; row(10 + k) = l.w[k]; }
#pragma unroll
    for (int k = 0; k < 4; ++k) { row(6 + k) = l.q[k]; row(13 + k) = l.d[k]; }
    if (mem) {
        auto mrow = [&](int k) -> float& { return elem(row_ptr(mem, ld, k), bo); };
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            mrow(k) = l.ip[k]; mrow(3 + k) = l.ia[k]; mrow(6 + k) = l.ir[k]; mrow(9 + k) = l.wprev[k];
        }
        mrow(12) = l.J;
    }
}

/* Tape slots: one block of kTapeRows x 64 floats per wave and step, a row
 * being 64 consecutive floats (one per lane).  `slot` is the block's base,
 * the same for the whole wave; rows 0-15 and 16-30 are addressed from two
 * scalar bases at immediate offsets (k x 256 bytes, within the 4 KiB range
 * of the instruction's offset field), and `lb` is the lane's byte offset. */
template <typename T>
struct TapeRows {
    T* lo;
    T* hi;
    __device__ __forceinline__ explicit TapeRows(T* slot) : lo(uniform(slot)), hi(uniform(slot + 16 * 64)) {}
    __device__ __forceinline__ T* row(int k) const { return k < 16 ? lo + k * 64 : hi + (k - 16) * 64; }
};

/* Step-start state of a tape slot: rows 0-25 (p, v, q, w, rotors, the three
 * integrals). */
__device__ __forceinline__ void store_tape(float* slot, uint32_t lb, const Agent& a) {
    const TapeRows<float> t(slot);
    auto row = [&](int k) -> float& { return elem(t.row(k), lb); };
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        row(k) = a.p[k]; row(3 + k) = a.v[k]; row(10 + k) = a.w[k];
        row(17 + k) = a.ip[k]; row(20 + k) = a.ia[k]; row(23 + k) = a.ir[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) { row(6 + k) = a.q[k]; row(13 + k) = a.d[k]; }
}

/* The controller's held command and branch decisions of a tape slot. */
__device__ __forceinline__ void store_tape_cmd(float* slot, uint32_t lb, const float dc[4], uint32_t bits) {
    const TapeRows<float> t(slot);
#pragma unroll
    for (int k = 0; k < 4; ++k) elem(t.row(kTapeCmd + k), lb) = dc[k];
    elem(t.row(kTapeBits), lb) = __uint_as_float(bits);
}

/* A tape slot: the step-start state (w_prev given by the caller; J and the
 * carries are not needed), the held command and the branch decisions. */
__device__ __forceinline__ void load_tape(const float* slot, uint32_t lb, const float wprev[3], Agent& a,
                                          float dc[4], uint32_t& bits) {
    const TapeRows<const float> t(slot);
    auto row = [&](int k) { return elem(t.row(k), lb); };
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        a.p[k] = row(k); a.v[k] = row(3 + k); a.w[k] = row(10 + k);
        a.ip[k] = row(17 + k); a.ia[k] = row(20 + k); a.ir[k] = row(23 + k);
        a.wprev[k] = wprev[k];
        a.p_lo[k] = a.v_lo[k] = a.ip_lo[k] = 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) { a.q[k] = row(6 + k); a.d[k] = row(13 + k); dc[k] = row(kTapeCmd + k); }
    bits = __float_as_uint(row(kTapeBits));
    a.J = a.J_lo = 0.0f;
}

/* Body rates at the start of a step (the w_prev of the next): rows 10-12
 * of a tape slot. */
__device__ __forceinline__ void load_tape_w(const float* slot, uint32_t lb, float w[3]) {
    const TapeRows<const float> t(slot);
#pragma unroll
    for (int k = 0; k < 3; ++k) w[k] = elem(t.row(10 + k), lb);
}

/* w_prev of step s of a segment: the body rates of step s - 1 on the tape,
 * or, for the segment's first step, the checkpoint's rows 26-28. */
__device__ __forceinline__ void step_wprev(const float* tape, int64_t tape_step, uint32_t lb, int s,
                                           const float* ckpt_seg, int64_t ld, uint32_t bo, float wprev[3]) {
    if (s > 0) {
        load_tape_w(tape + (int64_t)(s - 1) * tape_step, lb, wprev);
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) wprev[k] = elem(row_ptr(ckpt_seg, ld, 26 + k), bo);
    }
}

/* One recomputed forward step: its start state, held command and branch
 * decisions go to the tape slot, then the state advances (the forward
 * pass's own arithmetic, carries included, so the same bits). */
__device__ __forceinline__ void recompute_step(const TypeConst& c, const Limits& L, const Gains& g, Agent& a,
                                               const float wp[3], float* slot, uint32_t lb) {
    store_tape(slot, lb, a);
    float dc[4];
    uint32_t bits;
    controller<true, true>(c, L, g, a, wp, dc, &bits);
    store_tape_cmd(slot, lb, dc, bits);
    rk4_step(c, L, a, dc);
}

/*
 * Reverse sweep of one agent's closed-loop rollout of `steps` steps from
 * global step step0.  Checkpoint slot s (kCkptRows rows of stride ld: the
 * state, then its rounding carries; this agent's column at byte offset bo)
 * holds the state before call-relative step s*K.
 * Each segment is recomputed forward from its checkpoint with the
 * step-start states written to this wave's tape blocks (`tape` is the
 * wave's block of step 0, consecutive steps tape_step floats apart; lane
 * byte offset lb), then reversed step by step.
 * lam: cotangent of the final state on entry, of the initial state on
 * return; gk accumulates the gain cotangents.
 *
 * The loops run over the call's segments and slots (n_seg_all =
 * ceil(n_steps / K) and K, the same for every lane), and a lane skips the
 * iterations beyond its own step count.  All active lanes are therefore at
 * the same segment, slot and step, so checkpoint, tape and waypoint rows
 * are wave-uniform addresses even when step budgets differ between lanes.
 * Each reverse step loads its tape slot; the other resident wave covers
 * the load latency (holding the next slot in registers instead costs 30
 * registers and the second wave).
 */
__device__ __forceinline__ void agent_backward(const TypeConst& c, const Limits& L, const Gains& g,
                                               const float* ckpt, int64_t ld, uint32_t bo, int K,
                                               int n_seg_all, int steps, int64_t step0, const float* wp,
                                               int64_t cmd_ld, int n_epochs, int resample, float* tape,
                                               int64_t tape_step, uint32_t lb, AgentAdj& lam, float gk[9]) {
    const int n_seg = (steps + K - 1) / K;
    /* Waypoint epochs: global step k uses epoch min(k / resample, n_epochs - 1).
     * The epoch is divided out once per sweep of a segment and then tracked
     * across its boundaries, and the waypoint is reloaded only when the
     * (clamped) epoch changes. */
    const int64_t period = resample > 0 ? resample : INT64_MAX;
    int64_t cur_ep = -1;
    float wpv[3] = {0.0f, 0.0f, 0.0f};
    auto use_epoch = [&](int64_t e) {
        const int64_t ep = e < n_epochs - 1 ? e : (int64_t)n_epochs - 1;
        if (ep != cur_ep) {
#pragma unroll
            for (int i = 0; i < 3; ++i) wpv[i] = elem(uniform(wp + (ep * 3 + i) * cmd_ld), bo);
            cur_ep = ep;
        }
    };
    for (int seg = n_seg_all - 1; seg >= 0; --seg) {
        if (seg >= n_seg) continue;
        const int k_begin = seg * K;
        const int len = steps - k_begin < K ? steps - k_begin : K;
        const int64_t k0 = step0 + k_begin;        /* global index of the segment's first step */
        Agent a;
        load_rows(ckpt + (int64_t)seg * kCkptRows * ld, ld, bo, a, true);
        int64_t e = resample > 0 ? k0 / resample : 0;
        int64_t next = resample > 0 ? (e + 1) * period : INT64_MAX;   /* first step of epoch e + 1 */
        for (int s = 0; s < len; ++s) {
            if (k0 + s == next) { ++e; next += period; }
            use_epoch(e);
            recompute_step(c, L, g, a, wpv, tape + (int64_t)s * tape_step, lb);
        }
        /* reverse: start from the epoch of the segment's last step */
        e = resample > 0 ? (k0 + len - 1) / resample : 0;
        int64_t first = resample > 0 ? e * period : INT64_MIN;         /* first step of epoch e */
        const float* ck = ckpt + (int64_t)seg * kCkptRows * ld;
        for (int s = K - 1; s >= 0; --s) {
            if (s >= len) continue;
            if (k0 + s < first) { --e; first -= period; }
            Agent x;
            float dc[4], wprev[3];
            uint32_t bits;
            step_wprev(tape, tape_step, lb, s, ck, ld, bo, wprev);
            load_tape(tape + (int64_t)s * tape_step, lb, wprev, x, dc, bits);
            use_epoch(e);
            step_vjp(c, L, g, x, wpv, dc, bits, lam, gk);
        }
    }
}

/* Waypoint row of the current epoch (clamped to the last one), reloaded
 * only when the epoch changes. */
struct WaypointCache {
    const float* wp;
    int64_t cmd_ld;
    int n_epochs;
    uint32_t bo;
    int64_t cur = -1;
    float v[3] = {0.0f, 0.0f, 0.0f};
    __device__ __forceinline__ void use(int64_t e) {
        const int64_t ep = e < n_epochs - 1 ? e : (int64_t)n_epochs - 1;
        if (ep != cur) {
#pragma unroll
            for (int i = 0; i < 3; ++i) v[i] = elem(uniform(wp + (ep * 3 + i) * cmd_ld), bo);
            cur = ep;
        }
    }
};

/* The two halves of one segment of agent_backward, for a kernel that runs
 * them on different waves: the forward recomputation of segment `seg` from
 * its checkpoint into the tape, and the reverse sweep of a recomputed
 * segment.  Same operations, in the same order, as agent_backward. */
__device__ __forceinline__ void recompute_segment(const TypeConst& c, const Limits& L, const Gains& g,
                                                  const float* ckpt, int64_t ld, uint32_t bo, int K, int seg,
                                                  int steps, int64_t step0, int resample, WaypointCache& wc,
                                                  float* tape, int64_t tape_step, uint32_t lb) {
    const int64_t period = resample > 0 ? resample : INT64_MAX;
    const int k_begin = seg * K;
    const int len = steps - k_begin < K ? steps - k_begin : K;
    const int64_t k0 = step0 + k_begin;
    Agent a;
    load_rows(ckpt + (int64_t)seg * kCkptRows * ld, ld, bo, a, true);
    int64_t e = resample > 0 ? k0 / resample : 0;
    int64_t next = resample > 0 ? (e + 1) * period : INT64_MAX;
    for (int s = 0; s < len; ++s) {
        if (k0 + s == next) { ++e; next += period; }
        wc.use(e);
        recompute_step(c, L, g, a, wc.v, tape + (int64_t)s * tape_step, lb);
    }
}

__device__ __forceinline__ void reverse_segment(const TypeConst& c, const Limits& L, const Gains& g,
                                                const float* ckpt, int64_t ld, uint32_t bo, int K,
                                                int seg, int steps, int64_t step0, int resample,
                                                WaypointCache& wc, const float* tape, int64_t tape_step,
                                                uint32_t lb, AgentAdj& lam, float gk[9]) {
    const int64_t period = resample > 0 ? resample : INT64_MAX;
    const int k_begin = seg * K;
    const int len = steps - k_begin < K ? steps - k_begin : K;
    const int64_t k0 = step0 + k_begin;
    int64_t e = resample > 0 ? (k0 + len - 1) / resample : 0;
    int64_t first = resample > 0 ? e * period : INT64_MIN;
    const float* ck = ckpt + (int64_t)seg * kCkptRows * ld;
    for (int s = K - 1; s >= 0; --s) {
        if (s >= len) continue;
        if (k0 + s < first) { --e; first -= period; }
        Agent x;
        float dc[4], wprev[3];
        uint32_t bits;
        step_wprev(tape, tape_step, lb, s, ck, ld, bo, wprev);
        load_tape(tape + (int64_t)s * tape_step, lb, wprev, x, dc, bits);
        wc.use(e);
        step_vjp(c, L, g, x, wc.v, dc, bits, lam, gk);
    }
}

}  // namespace potato
