/*
 * quad_step.h -- per-agent FP32 arithmetic of one quadrotor time step, for
 * gfx950 kernels (one agent per lane, everything in registers).
 *
 * The physics follows Sec. II-B of the paper: eqs. (qd1)-(qd4) for the rigid
 * body, eq. (2) for rotor thrust/torque, eq. (3) for the allocation matrix,
 * classical RK4 for the discretisation, and a PID cascade ending in the
 * body-rate loop.  Differences from a literal transcription, all exact in
 * real arithmetic and chosen for FP32 accuracy or instruction count:
 *   - rotor speeds are carried as d = W - w_ref, and squared speeds as
 *     s = W^2 - w_ref^2 = d (2 w_ref + d), so the small speed differences
 *     that make the torques are not lost against a large W;
 *   - collective thrust over mass is F0 + (k_f/m) sum(s), F0 = 4 k_f w_ref^2/m,
 *     and the vertical acceleration is assembled as (F0 - g) + ... so that
 *     the hover cancellation thrust/m - g happens once, on the host;
 *   - the mixer uses the closed-form inverse G^-1 = G^T diag(1/|row|^2),
 *     exact because the rows of G are mutually orthogonal;
 *   - the rotor lag d' = (dc - d)/tau is linear with the command held, so the
 *     four RK4 stage values of d are dc + (d - dc) c_i with the RK4 stage
 *     polynomials c_i(z), z = -dt/tau, and the step ends at dc + (d - dc) R(z),
 *     R the RK4 stability polynomial (the numbers RK4 produces);
 *   - position obeys p' = v, so RK4 gives p + dt v + dt^2/6 (a1 + a2 + a3);
 *   - divisions by mass, inertia, tau_m and dt are multiplications by
 *     reciprocals precomputed per type;
 *   - the quaternion rate is evaluated as q o (0, w), and its factor 1/2
 *     rides on the RK4 step sizes (dt/4, dt/2, dt/12 instead of dt/2, dt,
 *     dt/6), a power of two, so the results are the same bits.
 * p, v, J and the position-loop integral are updated with a carried rounding
 * error (Fast2Sum), so long runs of nearly equal increments do not drift.
 *
 * Every forward function below turns floating-point contraction off and
 * places its fused multiply-adds explicitly: each kernel that inlines them
 * (plain, fused, type-indexed, adjoint recomputation) then executes the
 * same operations and produces the same bits.
 */
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace potato {

/* Constants of a car or fixed-wing type (vehicle kinds 1 and 2, see
 * vehicle_step.h), held in a type-table entry in place of a quadrotor's. */
struct VehConst {
    float inv_tau[3];     /* car: 1/tau_delta, 0, 0; wing: 1/tau_V, 1/tau_phi, 1/tau_gamma */
    float lim[3];         /* car: a_max, delta_max, 0; wing: 0, phi_max, gamma_max */
    float cruise;         /* cruise speed (m/s) */
    float rho, lam;       /* orbit radius (m) and direction (+1 counter-clockwise, -1 clockwise) */
    float lam_half_pi;    /* lam pi/2 */
    float k_orb_rho;      /* k_orb / rho: gain of the radial error in the course command */
    float k_head;         /* course error -> steering or bank */
    float k_hold;         /* car: speed-hold gain k_speed; wing: altitude-hold gain k_alt */
    float cd_m;           /* car: drag / m (1/s) */
    float inv_L, lr_L;    /* car: 1/wheelbase, l_r / wheelbase */
    float ff;             /* car: steering that holds the orbit, lam atan(L / sqrt(rho^2 - l_r^2)) */
    float inv_g_rho;      /* wing: 1 / (g rho) */
    float g;              /* wing: gravity */
};

/* Per-type constants, derived once on the host from potato_type_params and
 * rounded to FP32.  An entry holds a quadrotor's constants (kind 0) or a
 * car's or fixed-wing aircraft's (kinds 1, 2) in the same bytes. */
struct TypeConst {
    union {
        struct {
            float mass, inv_m, cd_m, ncd_m;       /* m, 1/m, c_d/m, -c_d/m */
            float Ix, Iy, Iz, iIx, iIy, iIz;      /* inertia and its inverse */
            float F0, F0_g, kf_m;                 /* 4 k_f w_ref^2/m, F0 - g, k_f/m */
            float F0_2, kf_m2;                    /* 2 F0, 2 k_f/m (exact doublings) */
            float kf_ls, kf_lc, km;               /* k_f L sin(a), k_f L cos(a), k_m */
            float ax, ay, az;                     /* k_f L sin(a)/Ixx, k_f L cos(a)/Iyy, k_m/Izz */
            float gx, gy, gz;                     /* (Izz-Iyy)/Ixx, (Ixx-Izz)/Iyy, (Iyy-Ixx)/Izz */
            float w_ref, two_w, four_w2;          /* w_ref, 2 w_ref, 4 w_ref^2 */
            float inv_tau;                        /* 1 / tau_m */
            float mix_x, mix_y, mix_z;            /* 1/(4 L sin a), 1/(4 L cos a), k_f/(4 k_m) */
            float f_max, inv_kf;                  /* k_f w_max^2, 1/k_f */
            float gains[9];
        };
        VehConst veh;
    };
    int32_t budget;
    int16_t kind;                                 /* 0 quadrotor, 1 car, 2 fixed wing */
    int16_t group;                                /* class for grouping agents within a block */
};
static_assert(sizeof(TypeConst) == 44 * 4, "type table entry: 42 constants, budget, kind and group");

enum { KIND_QUAD = 0, KIND_CAR = 1, KIND_WING = 2 };

/* Controller limits and the time step, shared by all agents of a launch. */
struct Limits {
    float g, r_sat, r_sat2, ipos_max, iatt_max, irate_max, az_min;
    float dt, half_dt, dt6, inv_dt, dt2_6;   /* dt, dt/2, dt/6, 1/dt, dt^2/6 */
    float quarter_dt, dt12;                  /* half_dt/2, dt6/2 (exact halvings) */
};

struct Gains {
    float kpp, kip, kdp, kpa, kia, kda, kpr, kir, kdr;
    float kdr_dt;                         /* kdr / dt, set once per agent and launch */
};

/* 17 integrated rows + running cost, the controller memory, and the
 * rounding carries of p, v, J and the position-loop integral. */
struct Agent {
    float p[3], v[3], q[4], w[3], d[4];   /* d = rotor speed - w_ref */
    float J;
    float ip[3], ia[3], ir[3], wprev[3];
    float p_lo[3], v_lo[3], J_lo, ip_lo[3];
};

/* Element of a structure-of-arrays row.  `row` is the same address in every
 * lane of the wave (it stays in scalar registers) and `boff` is the lane's
 * byte offset into the row (agent index times the element size), below
 * 2^32.  Each access is then a single global load or store with a scalar
 * base and a 32-bit vector offset, and no 64-bit address per row occupies
 * vector registers. */
template <typename T>
__device__ __forceinline__ T& elem(T* row, uint32_t boff) {
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return *reinterpret_cast<T*>(reinterpret_cast<B*>(row) + boff);
}

/* `p`, a pointer that is the same in every active lane, marked as such: the
 * compiler then keeps it in scalar registers and addresses with it as the
 * scalar base, instead of folding a lane's offset into a 64-bit vector
 * address per row (which costs two vector registers per row).  Only for
 * values that are truly uniform over the active lanes. */
template <typename T>
__device__ __forceinline__ T* uniform(T* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    /* the rebuilt address is device (global) memory: passing it through the
     * global address space keeps the accesses global rather than flat */
    typedef __attribute__((address_space(1))) char gchar;
    return (T*)(gchar*)(((uint64_t)hi << 32) | lo);
}

/* Type index of agent i, clamped to the table: an index >= n_types reads
 * as the last type, so a bad index never addresses past the table. */
__device__ __forceinline__ uint32_t type_entry(const uint8_t* type, uint32_t i, int n_types) {
    const uint32_t t = type[i];
    const uint32_t last = (uint32_t)(n_types - 1);
    return t < last ? t : last;
}

/* Entry j of a processing order over n agents, clamped to [0, n): an entry
 * outside the range (a caller's order that is not a permutation) reads as
 * the last agent, so no lane addresses past the state rows. */
__device__ __forceinline__ uint32_t order_entry(const int32_t* perm, uint32_t j, int64_t n) {
    const uint32_t a = (uint32_t)elem(perm, j << 2);
    const uint32_t last = (uint32_t)(n - 1);
    return a < last ? a : last;
}

/* Rows per step of the adjoint's recomputation tape: the step-start state
 * without its cost and previous body rates (26 rows: p, v, q, w, rotors,
 * the three integrals), the rotor command the controller held through the
 * step (4) and the controller's branch decisions (1, bits as a float). */
constexpr int kTapeRows = 31;
constexpr int kTapeCmd = 26;      /* first row of the held command */
constexpr int kTapeBits = 30;     /* row of the branch decisions */

/* Branch decisions of one controller evaluation, recorded by the forward
 * pass so that the reverse sweep differentiates exactly the branches it
 * took (bit set = condition true). */
enum : uint32_t {
    kBitSat = 1u << 0,            /* position error saturated to r_sat */
    kBitIp = 1u << 1,             /* bits 1-3: position integral inside its clamp, per axis */
    kBitAz = 1u << 4,             /* vertical acceleration raised to its floor */
    kBitSgn = 1u << 5,            /* error quaternion flipped to the short arc */
    kBitIa = 1u << 6,             /* bits 6-8: attitude integral inside its clamp */
    kBitIr = 1u << 9,             /* bits 9-11: rate integral inside its clamp */
    kBitRotor = 1u << 12          /* bits 12-15: rotor thrust in (0, f_max] (speed differentiable) */
};

#define POTATO_FMA(a, b, c) __builtin_fmaf((a), (b), (c))

/* x += inc with the rounding error carried in lo (Fast2Sum, Dekker 1971):
 * the low part is added back into the next increment.  Without CARRY the
 * update is the plain rounded sum and lo is left alone. */
template <bool CARRY>
__device__ __forceinline__ void add_carry(float& x, float& lo, float inc) {
#pragma clang fp contract(off)
    if (CARRY) {
        const float y = inc + lo;
        const float s = x + y;
        lo = y - (s - x);
        x = s;
    } else {
        x = x + inc;
    }
}

/* clamp(x, lo, hi) for lo <= hi (one v_med3_f32). */
__device__ __forceinline__ float clampf_(float x, float lo, float hi) {
    return __builtin_amdgcn_fmed3f(x, lo, hi);
}

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float sqrt_fast(float x) { return __builtin_amdgcn_sqrtf(x); }

/* Body z axis in the inertial frame: third column of R(q), unit-norm form
 * (eq. qd2 with thrust along body z). */
__device__ __forceinline__ void body_z(const float q[4], float bz[3]) {
#pragma clang fp contract(off)
    bz[0] = 2.0f * POTATO_FMA(q[0], q[2], q[1] * q[3]);
    bz[1] = 2.0f * POTATO_FMA(q[2], q[3], -(q[0] * q[1]));
    bz[2] = POTATO_FMA(-2.0f, POTATO_FMA(q[1], q[1], q[2] * q[2]), 1.0f);
}

/* Rates of v and w at rotor deviations d (eqs. 2, 3, qd2, qd4), and
 * dq = q o (0, w), twice the quaternion rate of eq. (qd3): the factor 1/2
 * is carried by the RK4 step sizes instead (exactly, as a power of two).
 * Returns sum_i s_i (collective thrust and cost rate follow from it). */
__device__ __forceinline__ float rates(const TypeConst& c, const float v[3], const float q[4],
                                       const float w[3], const float d[4], float dv[3], float dq[4],
                                       float dw[3]) {
#pragma clang fp contract(off)
    /* eq. (2) with s_i = W_i^2 - w_ref^2 */
    float s[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) s[i] = POTATO_FMA(d[i], d[i], c.two_w * d[i]);
    const float A = s[0] - s[1], B = s[3] - s[2];
    const float P01 = s[0] + s[1], P23 = s[2] + s[3];
    const float ssum = P01 + P23;
    /* eq. (qd2) + drag: (f_c/m) R(q) z - (c_d/m) v - g z */
    const float ftm2 = POTATO_FMA(c.kf_m2, ssum, c.F0_2);
    const float bx2 = POTATO_FMA(q[0], q[2], q[1] * q[3]);
    const float by2 = POTATO_FMA(q[2], q[3], -(q[0] * q[1]));
    const float x2y2 = POTATO_FMA(q[1], q[1], q[2] * q[2]);
    dv[0] = POTATO_FMA(ftm2, bx2, c.ncd_m * v[0]);
    dv[1] = POTATO_FMA(ftm2, by2, c.ncd_m * v[1]);
    dv[2] = POTATO_FMA(c.ncd_m, v[2], POTATO_FMA(-ftm2, x2y2, POTATO_FMA(c.kf_m, ssum, c.F0_g)));
    /* eq. (qd3) without its factor 1/2: q o (0, w) */
    dq[0] = -POTATO_FMA(q[3], w[2], POTATO_FMA(q[2], w[1], q[1] * w[0]));
    dq[1] = POTATO_FMA(-q[3], w[1], POTATO_FMA(q[2], w[2], q[0] * w[0]));
    dq[2] = POTATO_FMA(-q[1], w[2], POTATO_FMA(q[3], w[0], q[0] * w[1]));
    dq[3] = POTATO_FMA(-q[2], w[0], POTATO_FMA(q[1], w[1], q[0] * w[2]));
    /* eq. (3) torques and eq. (qd4): w' = I^-1 (tau - w x I w) */
    dw[0] = POTATO_FMA(-c.gx, w[1] * w[2], c.ax * (A + B));
    dw[1] = POTATO_FMA(-c.gy, w[2] * w[0], c.ay * (P23 - P01));
    dw[2] = POTATO_FMA(-c.gz, w[0] * w[1], c.az * (A - B));
    return ssum;
}

/* Rate of the integrated rows for held rotor command dc (relative to
 * w_ref): the general form, used where a single derivative is needed. */
__device__ __forceinline__ void derivative(const TypeConst& c, const float v[3], const float q[4],
                                           const float w[3], const float d[4], const float dc[4],
                                           float dv[3], float dq[4], float dw[3], float dd[4],
                                           float& dJ) {
#pragma clang fp contract(off)
    const float ssum = rates(c, v, q, w, d, dv, dq, dw);
#pragma unroll
    for (int i = 0; i < 4; ++i) dq[i] *= 0.5f;
#pragma unroll
    for (int i = 0; i < 4; ++i) dd[i] = (dc[i] - d[i]) * c.inv_tau;
    dJ = c.four_w2 + ssum;
}

/* Position -> attitude -> body-rate PID cascade and mixer, evaluated once
 * per step on the step-start state; returns rotor commands relative to
 * w_ref and updates the controller memory.  CARRY: the position-loop
 * integral keeps its rounding carry in a.ip_lo.  BITS: the branch
 * decisions go to *bits (kBit*; comparisons only, the arithmetic is the
 * same). */
template <bool CARRY = true, bool BITS = false>
__device__ __forceinline__ void controller(const TypeConst& c, const Limits& L, const Gains& k,
                                           Agent& a, const float wp[3], float dc[4],
                                           uint32_t* bits = nullptr) {
#pragma clang fp contract(off)
    /* position loop: error saturated to radius r_sat */
    float e[3] = {wp[0] - a.p[0], wp[1] - a.p[1], wp[2] - a.p[2]};
    const float n2 = POTATO_FMA(e[2], e[2], POTATO_FMA(e[1], e[1], e[0] * e[0]));
    const float sc = n2 > L.r_sat2 ? L.r_sat * rsq(n2) : 1.0f;
    uint32_t b = n2 > L.r_sat2 ? kBitSat : 0u;
    float acc[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        e[i] *= sc;
        /* integral with carried rounding error, clamped (carry cleared at a bound) */
        const float y = CARRY ? POTATO_FMA(e[i], L.dt, a.ip_lo[i]) : e[i] * L.dt;
        const float s = a.ip[i] + y;
        const float cl = clampf_(s, -L.ipos_max, L.ipos_max);
        if (CARRY) {
            const float lo = y - (s - a.ip[i]);
            a.ip_lo[i] = cl == s ? lo : 0.0f;
        }
        if (BITS && cl == s) b |= kBitIp << i;
        a.ip[i] = cl;
        acc[i] = POTATO_FMA(-k.kdp, a.v[i], POTATO_FMA(k.kip, cl, k.kpp * e[i]));
    }
    if (BITS && acc[2] + L.g < L.az_min) b |= kBitAz;
    acc[2] = fmaxf(acc[2] + L.g, L.az_min);

    /* collective thrust: commanded acceleration along the current body z */
    float bz[3];
    body_z(a.q, bz);
    const float fc = c.mass * POTATO_FMA(acc[2], bz[2], POTATO_FMA(acc[1], bz[1], acc[0] * bz[0]));

    /* desired attitude: shortest rotation of z onto the thrust direction,
     * q_des ~ (1 + n_z, -n_y, n_x, 0), whose squared norm is 2 (1 + n_z) */
    const float ra = rsq(POTATO_FMA(acc[2], acc[2], POTATO_FMA(acc[1], acc[1], acc[0] * acc[0])));
    const float nx = acc[0] * ra, ny = acc[1] * ra, nz = acc[2] * ra;
    const float qr0 = 1.0f + nz;
    const float rq = rsq(qr0 + qr0);
    const float qd0 = qr0 * rq, qd1 = -(ny * rq), qd2 = nx * rq;

    /* attitude loop on conj(q) o q_des (short arc) */
    const float* q = a.q;
    const float ew = POTATO_FMA(q[2], qd2, POTATO_FMA(q[1], qd1, q[0] * qd0));
    const float ex = POTATO_FMA(q[3], qd2, POTATO_FMA(-q[1], qd0, q[0] * qd1));
    const float ey = POTATO_FMA(-q[3], qd1, POTATO_FMA(-q[2], qd0, q[0] * qd2));
    const float ez = POTATO_FMA(-q[3], qd0, POTATO_FMA(-q[1], qd2, q[2] * qd1));
    const float sg = ew < 0.0f ? -2.0f : 2.0f;
    if (BITS && ew < 0.0f) b |= kBitSgn;
    const float eatt[3] = {sg * ex, sg * ey, sg * ez};
    float alpha[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float pa = POTATO_FMA(eatt[i], L.dt, a.ia[i]);
        a.ia[i] = clampf_(pa, -L.iatt_max, L.iatt_max);
        if (BITS && a.ia[i] == pa) b |= kBitIa << i;
        const float wdes = POTATO_FMA(-k.kda, a.w[i], POTATO_FMA(k.kia, a.ia[i], k.kpa * eatt[i]));
        /* body-rate loop, derivative on the measured rate */
        const float erate = wdes - a.w[i];
        const float pr = POTATO_FMA(erate, L.dt, a.ir[i]);
        a.ir[i] = clampf_(pr, -L.irate_max, L.irate_max);
        if (BITS && a.ir[i] == pr) b |= kBitIr << i;
        alpha[i] = POTATO_FMA(-k.kdr_dt, a.w[i] - a.wprev[i], POTATO_FMA(k.kir, a.ir[i], k.kpr * erate));
        a.wprev[i] = a.w[i];
    }
    /* torque for the desired angular acceleration, eq. (qd4) inverted */
    const float Iwx = c.Ix * a.w[0], Iwy = c.Iy * a.w[1], Iwz = c.Iz * a.w[2];
    const float tx = POTATO_FMA(c.Ix, alpha[0], POTATO_FMA(a.w[1], Iwz, -(a.w[2] * Iwy)));
    const float ty = POTATO_FMA(c.Iy, alpha[1], POTATO_FMA(a.w[2], Iwx, -(a.w[0] * Iwz)));
    const float tz = POTATO_FMA(c.Iz, alpha[2], POTATO_FMA(a.w[0], Iwy, -(a.w[1] * Iwx)));

    /* mixer: f = G^-1 [fc, tau], saturate, invert eq. (2) */
    const float f4 = 0.25f * fc;
    const float X = tx * c.mix_x, Y = ty * c.mix_y, Z = tz * c.mix_z;
    const float fpz = f4 + Z, fmz = f4 - Z, xmy = X - Y, xpy = X + Y;
    const float f[4] = {fpz + xmy, fmz - xpy, fpz - xmy, fmz + xpy};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float fi = clampf_(f[i], 0.0f, c.f_max);
        if (BITS && f[i] > 0.0f && f[i] <= c.f_max) b |= kBitRotor << i;
        dc[i] = sqrt_fast(fi * c.inv_kf) - c.w_ref;
    }
    if (BITS) *bits = b;
}

/* Classical RK4 with the command held, then quaternion renormalisation.
 * CARRY: p, v and J keep their rounding carries in a.p_lo, a.v_lo, a.J_lo. */
template <bool CARRY = true>
__device__ __forceinline__ void rk4_step(const TypeConst& c, const Limits& L, Agent& a,
                                         const float dc[4]) {
#pragma clang fp contract(off)
    /* RK4 stage polynomials of the linear rotor lag, z = -dt / tau */
    const float z = -(L.dt * c.inv_tau);
    const float hz = 0.5f * z;
    const float c2 = 1.0f + hz;
    const float c3 = POTATO_FMA(hz, c2, 1.0f);
    const float c4 = POTATO_FMA(z, c3, 1.0f);
    const float cR = POTATO_FMA(z * (1.0f / 6.0f), ((1.0f + (c2 + c2)) + (c3 + c3)) + c4, 1.0f);
    float e[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) e[i] = a.d[i] - dc[i];

    float kv[3], kq[4], kw[3];            /* stage rates */
    float av[3], aq[4], aw[3], A3[3];     /* weighted sums; A3 = a1 + a2 + a3 */
    float sv[3], sq[4], sw[3], sd[4];     /* stage state */
    float ss, ass;

    /* stage 1 */
    ss = rates(c, a.v, a.q, a.w, a.d, kv, kq, kw);
#pragma unroll
    for (int i = 0; i < 3; ++i) { av[i] = kv[i]; aw[i] = kw[i]; A3[i] = kv[i]; }
#pragma unroll
    for (int i = 0; i < 4; ++i) aq[i] = kq[i];
    ass = ss;
    /* stage 2 */
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        sv[i] = POTATO_FMA(L.half_dt, kv[i], a.v[i]);
        sw[i] = POTATO_FMA(L.half_dt, kw[i], a.w[i]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) { sq[i] = POTATO_FMA(L.quarter_dt, kq[i], a.q[i]); sd[i] = POTATO_FMA(e[i], c2, dc[i]); }
    ss = rates(c, sv, sq, sw, sd, kv, kq, kw);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        av[i] = POTATO_FMA(2.0f, kv[i], av[i]);
        aw[i] = POTATO_FMA(2.0f, kw[i], aw[i]);
        A3[i] += kv[i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) aq[i] = POTATO_FMA(2.0f, kq[i], aq[i]);
    ass = POTATO_FMA(2.0f, ss, ass);
    /* stage 3 */
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        sv[i] = POTATO_FMA(L.half_dt, kv[i], a.v[i]);
        sw[i] = POTATO_FMA(L.half_dt, kw[i], a.w[i]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) { sq[i] = POTATO_FMA(L.quarter_dt, kq[i], a.q[i]); sd[i] = POTATO_FMA(e[i], c3, dc[i]); }
    ss = rates(c, sv, sq, sw, sd, kv, kq, kw);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        av[i] = POTATO_FMA(2.0f, kv[i], av[i]);
        aw[i] = POTATO_FMA(2.0f, kw[i], aw[i]);
        A3[i] += kv[i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) aq[i] = POTATO_FMA(2.0f, kq[i], aq[i]);
    ass = POTATO_FMA(2.0f, ss, ass);
    /* stage 4 */
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        sv[i] = POTATO_FMA(L.dt, kv[i], a.v[i]);
        sw[i] = POTATO_FMA(L.dt, kw[i], a.w[i]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) { sq[i] = POTATO_FMA(L.half_dt, kq[i], a.q[i]); sd[i] = POTATO_FMA(e[i], c4, dc[i]); }
    ss = rates(c, sv, sq, sw, sd, kv, kq, kw);
    ass += ss;

    /* combine: p with dt v + dt^2/6 (a1 + a2 + a3), the rest dt/6 (k1 + 2k2 + 2k3 + k4)
     * (dt/12 for q, whose stage rates are doubled) */
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        add_carry<CARRY>(a.p[i], a.p_lo[i], POTATO_FMA(L.dt2_6, A3[i], L.dt * a.v[i]));
        add_carry<CARRY>(a.v[i], a.v_lo[i], L.dt6 * (av[i] + kv[i]));
        a.w[i] = POTATO_FMA(L.dt6, aw[i] + kw[i], a.w[i]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        a.q[i] = POTATO_FMA(L.dt12, aq[i] + kq[i], a.q[i]);
        a.d[i] = POTATO_FMA(e[i], cR, dc[i]);
    }
    add_carry<CARRY>(a.J, a.J_lo, POTATO_FMA(L.dt6, ass, L.dt * c.four_w2));

    const float r = rsq(POTATO_FMA(a.q[3], a.q[3],
                        POTATO_FMA(a.q[2], a.q[2], POTATO_FMA(a.q[1], a.q[1], a.q[0] * a.q[0]))));
#pragma unroll
    for (int i = 0; i < 4; ++i) a.q[i] *= r;
}

}  // namespace potato
