/*
 * oracle.cpp -- plain, slow, FP64 CPU reference of the batched quadrotor
 * time step of "Potato" (arXiv 2308.12698).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing but the test-suite, the smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no
 * source, header, constant or helper with the HIP kernels; the two meet only
 * through the seeded input generator.
 *
 * What it computes, per agent and per step (scalar double, one agent at a
 * time, no blocking or fusion):
 *   - rigid-body model, eqs. (qd1)-(qd4) of Sec. II-B, with gravity
 *     [0, 0, -g] in the ENU inertial frame and thrust along body z;
 *   - rotor model f_i = k_t W_i^2, tau_i = k_q W_i^2, eq. (2);
 *   - control allocation [f_c, tau] = G [f_1..f_4], eq. (3) and the G
 *     matrix printed beneath it; the mixer solves that system;
 *   - classical fourth-order Runge-Kutta discretisation (end of Sec. II-B);
 *   - a PID cascade whose innermost loop is the body-rate controller the
 *     paper names at the end of Sec. II-B (outer position and attitude loops
 *     are this project's reading, listed in the design notes);
 *   - first-order rotor lag and linear drag (workload definition, not in the
 *     paper).
 * The paper batches agents as tensors (Sec. I, Fig. 1); batching changes
 * no agent's arithmetic, so the reference is simply a loop over agents.
 *
 * The step, controller and dynamics are templates on the scalar type so the
 * same source runs in double (values), in forward-mode dual numbers
 * (Jacobians of the rollout) and in an operation-counting scalar (the
 * algorithmic flop count per agent-step).
 *
 * Pins (tests/test_oracle_pins.py, tests/test_oracle_grad.py): closed
 * forms of the dynamics, conservation laws, RK4 order, the allocation
 * geometry, linearised closed-loop step responses, saturated regimes and an
 * independent rotation-matrix formulation of large coupled manoeuvres;
 * dual numbers against central differences.  Parity unpinned: the outer
 * position and attitude loops as a definition (the paper delegates them to
 * a cited work); the tests pin this implementation of the project's
 * reading of them, not the reading.
 */
#include <cmath>
#include <cstdint>
#include <cstring>
#include <omp.h>

namespace {

/* ------------------------------------------------------------------ */
/* Scalar types                                                         */
/* ------------------------------------------------------------------ */

inline double val(double x) { return x; }
inline double sqrt_(double x) { return std::sqrt(x); }

/* Forward-mode dual number with N tangent directions. */
template <int N>
struct Dual {
    double v;
    double d[N];
    Dual() : v(0.0) { for (int i = 0; i < N; ++i) d[i] = 0.0; }
    Dual(double x) : v(x) { for (int i = 0; i < N; ++i) d[i] = 0.0; }
};
template <int N> inline double val(const Dual<N>& a) { return a.v; }
template <int N> inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r(a.v + b.v); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r(a.v - b.v); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a) {
    Dual<N> r(-a.v); for (int i = 0; i < N; ++i) r.d[i] = -a.d[i]; return r; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r(a.v * b.v); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r(a.v / b.v);
    for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
    return r; }
template <int N> inline Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> inline Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> inline Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, double b) { return a * Dual<N>(b); }
template <int N> inline Dual<N> operator*(double a, const Dual<N>& b) { return Dual<N>(a) * b; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, double b) { return a / Dual<N>(b); }
template <int N> inline Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }
/* sqrt'(0) is taken as 0: a rotor command clamped to zero thrust has no
 * sensitivity, and the clamp has already zeroed the incoming tangent. */
template <int N> inline Dual<N> sqrt_(const Dual<N>& a) {
    Dual<N> r(std::sqrt(a.v));
    double s = r.v > 0.0 ? 0.5 / r.v : 0.0;
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * s;
    return r; }

/* Operation-counting scalar (single-threaded use only).
 *
 * Forward count: the floating-point operations one evaluation performs, by
 * kind, with three rules that keep the count to the arithmetic the model
 * needs rather than that of its textbook matrix forms:
 *   - a value built from the literal 0 is a structural zero: a product with
 *     it is again a structural zero and costs nothing, and adding it,
 *     subtracting it or subtracting from it costs nothing (the zero scalar
 *     part of (0, w) in eq. (qd3), the zero last component of the
 *     desired-attitude quaternion);
 *   - a product with an entry of G (eq. 3) that is exactly 1 or -1 costs
 *     nothing (G's row of ones; see gmul);
 *   - a sign flip costs nothing (it is an operand modifier).
 * Inputs (state, controller memory, gains) are marked as variables; the
 * count assumes none of them is exactly 0 or +-1.
 *
 * Reverse count `rev`: the flops of the reverse sweep (vector-Jacobian
 * product) that accumulates the cotangents of each counted operation's
 * variable operands, by the elementary rules of reverse-mode
 * differentiation (for z = a o b and cotangent zb):
 *   a + b, a - b:  ab += zb, bb +-= zb            1 add per variable operand
 *   a * b:         ab += zb * b, bb += zb * a      1 mul + 1 add per variable operand
 *   a / b:         ab += zb / b                    1 div + 1 add if a is a variable
 *                  bb -= zb * z / b                1 mul + 1 div + 1 add if b is
 *   sqrt(a):       ab += 0.5 * (zb / z)            1 div + 1 mul + 1 add
 * A product with an entry +-1 of G passes its cotangent on (1 add); sign
 * flips and comparisons cost nothing. */
struct OpCount { int64_t add, mul, div, sqrt, cmp, rev; };
OpCount g_ops;
struct Cnt {
    double v;
    bool zero, var;
    Cnt() : v(0), zero(true), var(false) {}
    Cnt(double x) : v(x), zero(x == 0.0), var(false) {}
    static Cnt input(double x) { Cnt c(x); c.zero = false; c.var = true; return c; }
    static Cnt result(double x, bool var) { Cnt c(x); c.zero = false; c.var = var; return c; }
};
inline double val(const Cnt& a) { g_ops.cmp++; return a.v; }
inline Cnt operator-(Cnt a) { a.v = -a.v; return a; }   /* sign flip: a modifier, not an op */
inline Cnt operator+(Cnt a, Cnt b) {
    if (a.zero) return b;
    if (b.zero) return a;
    g_ops.add++;
    g_ops.rev += (int)a.var + (int)b.var;
    return Cnt::result(a.v + b.v, a.var || b.var);
}
inline Cnt operator-(Cnt a, Cnt b) {
    if (b.zero) return a;
    if (a.zero) return -b;
    g_ops.add++;
    g_ops.rev += (int)a.var + (int)b.var;
    return Cnt::result(a.v - b.v, a.var || b.var);
}
inline Cnt operator*(Cnt a, Cnt b) {
    if (a.zero || b.zero) return Cnt(0.0);
    g_ops.mul++;
    g_ops.rev += 2 * ((int)a.var + (int)b.var);
    return Cnt::result(a.v * b.v, a.var || b.var);
}
inline Cnt operator/(Cnt a, Cnt b) {
    if (a.zero) return Cnt(0.0);
    g_ops.div++;
    g_ops.rev += (a.var ? 2 : 0) + (b.var ? 3 : 0);
    return Cnt::result(a.v / b.v, a.var || b.var);
}
inline Cnt operator+(Cnt a, double b) { return a + Cnt(b); }
inline Cnt operator+(double a, Cnt b) { return Cnt(a) + b; }
inline Cnt operator-(Cnt a, double b) { return a - Cnt(b); }
inline Cnt operator-(double a, Cnt b) { return Cnt(a) - b; }
inline Cnt operator*(Cnt a, double b) { return a * Cnt(b); }
inline Cnt operator*(double a, Cnt b) { return Cnt(a) * b; }
inline Cnt operator/(Cnt a, double b) { return a / Cnt(b); }
inline Cnt operator/(double a, Cnt b) { return Cnt(a) / b; }
inline Cnt sqrt_(Cnt a) {
    g_ops.sqrt++;
    if (a.var) g_ops.rev += 3;
    return Cnt::result(std::sqrt(a.v), a.var);
}

/* clamp(x, lo, hi) = x < lo ? lo : (x > hi ? hi : x); the derivative is that
 * of the branch taken (1 inside [lo, hi], 0 outside). */
template <class T> inline T clamp_(const T& x, double lo, double hi) {
    if (val(x) < lo) return T(lo);
    if (val(x) > hi) return T(hi);
    return x;
}

/* Product of an entry of the allocation matrix G (eq. 3) with a rotor
 * thrust.  Plain multiplication; the counting scalar treats an entry of
 * exactly +-1 (G's first row) as free, since the collective thrust is the
 * plain sum of the rotor thrusts. */
template <class T> inline T gmul(double g, const T& f) { return g * f; }
inline Cnt gmul(double g, const Cnt& f) {
    if (g != 1.0 && g != -1.0) return g * f;
    if (f.var) g_ops.rev += 1;
    Cnt r = f;
    r.v = g * f.v;
    return r;
}

/* ------------------------------------------------------------------ */
/* Parameters                                                           */
/* ------------------------------------------------------------------ */

}  // namespace

extern "C" {

/* One airframe type, FP64.  Field order is part of the ctypes binding. */
typedef struct {
    double mass, Ixx, Iyy, Izz, arm, alpha, k_f, k_m, tau_m, drag, w_max, w_ref;
    double gains[9];          /* kpp kip kdp kpa kia kda kpr kir kdr */
    int64_t step_budget;      /* steps an agent of this type may take */
} oracle_type;

typedef struct {
    double g, r_sat, ipos_max, iatt_max, irate_max, az_min_frac;
} oracle_globals;

}  // extern "C"

namespace {

/* ODE state indices (absolute rotor speeds, running cost last). */
enum { P = 0, V = 3, Q = 6, W = 10, M = 13, JC = 17, NX = 18 };
/* Controller memory indices. */
enum { IP = 0, IA = 3, IR = 6, WPREV = 9, NMEM = 12 };

struct TypeData {
    oracle_type t;
    double G[4][4];      /* control allocation matrix, eq. (3) */
    double Ginv[4][4];   /* its inverse, by Gauss-Jordan elimination */
};

/* The allocation matrix printed under eq. (3): rows (f_c, tau_x, tau_y,
 * tau_z), columns rotors 1..4. */
void build_G(const oracle_type& t, double G[4][4]) {
    const double ls = t.arm * std::sin(t.alpha), lc = t.arm * std::cos(t.alpha);
    const double kr = t.k_m / t.k_f;
    const double rows[4][4] = {
        {1.0, 1.0, 1.0, 1.0},
        {ls, -ls, -ls, ls},
        {-lc, -lc, lc, lc},
        {kr, -kr, kr, -kr}};
    std::memcpy(G, rows, sizeof(rows));
}

/* Inverse of a 4x4 matrix by Gauss-Jordan elimination with partial
 * pivoting.  Returns false if singular. */
bool invert4(const double A[4][4], double Ainv[4][4]) {
    double a[4][8];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 8; ++j) a[i][j] = j < 4 ? A[i][j] : (j - 4 == i ? 1.0 : 0.0);
    for (int c = 0; c < 4; ++c) {
        int piv = c;
        for (int r = c + 1; r < 4; ++r)
            if (std::fabs(a[r][c]) > std::fabs(a[piv][c])) piv = r;
        if (a[piv][c] == 0.0) return false;
        for (int j = 0; j < 8; ++j) { double tmp = a[c][j]; a[c][j] = a[piv][j]; a[piv][j] = tmp; }
        const double inv = 1.0 / a[c][c];
        for (int j = 0; j < 8; ++j) a[c][j] *= inv;
        for (int r = 0; r < 4; ++r) {
            if (r == c) continue;
            const double f = a[r][c];
            for (int j = 0; j < 8; ++j) a[r][j] -= f * a[c][j];
        }
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) Ainv[i][j] = a[i][j + 4];
    return true;
}

bool make_type(const oracle_type& t, TypeData& td) {
    td.t = t;
    build_G(t, td.G);
    return invert4(td.G, td.Ginv);
}

/* ------------------------------------------------------------------ */
/* Kinematics helpers                                                   */
/* ------------------------------------------------------------------ */

/* Hamilton product a o b, scalar-first quaternions (eq. qd3 uses "o"). */
template <class T>
void quat_mul(const T a[4], const T b[4], T r[4]) {
    r[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    r[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    r[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    r[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

/* Third column of the rotation matrix R(q) of a unit quaternion, i.e. the
 * body z axis expressed in the inertial frame (eq. qd2 with B f_u along z).
 * Applied as-is to the non-unit quaternions of intermediate RK4 stages. */
template <class T>
void body_z_axis(const T q[4], T z[3]) {
    z[0] = 2.0 * (q[1] * q[3] + q[0] * q[2]);
    z[1] = 2.0 * (q[2] * q[3] - q[0] * q[1]);
    z[2] = 1.0 - 2.0 * (q[1] * q[1] + q[2] * q[2]);
}

/* ------------------------------------------------------------------ */
/* Dynamics: right-hand side of eqs. (qd1)-(qd4) plus rotor lag and cost  */
/* ------------------------------------------------------------------ */

template <class T>
void derivative(const TypeData& td, double g, const T x[NX], const T Wcmd[4], T dx[NX]) {
    const oracle_type& t = td.t;
    /* eq. (2): per-rotor thrust from the squared speeds (which also give the
     * rate of the running cost below) */
    T w2[4], f[4];
    for (int i = 0; i < 4; ++i) {
        w2[i] = x[M + i] * x[M + i];
        f[i] = t.k_f * w2[i];
    }
    /* eq. (3): collective thrust and body torques */
    T u[4];
    for (int r = 0; r < 4; ++r)
        u[r] = gmul(td.G[r][0], f[0]) + gmul(td.G[r][1], f[1]) + gmul(td.G[r][2], f[2]) +
               gmul(td.G[r][3], f[3]);
    const T fc = u[0];
    const T tau[3] = {u[1], u[2], u[3]};
    /* eq. (qd1) */
    for (int i = 0; i < 3; ++i) dx[P + i] = x[V + i];
    /* eq. (qd2) plus linear drag -(c_d/m) v */
    T bz[3];
    body_z_axis(&x[Q], bz);
    const T fcm = fc / t.mass;
    for (int i = 0; i < 3; ++i) dx[V + i] = fcm * bz[i] - (t.drag / t.mass) * x[V + i];
    dx[V + 2] = dx[V + 2] - g;
    /* eq. (qd3): q' = 1/2 q o [0, w] */
    const T wq[4] = {T(0.0), x[W + 0], x[W + 1], x[W + 2]};
    T qw[4];
    quat_mul(&x[Q], wq, qw);
    for (int i = 0; i < 4; ++i) dx[Q + i] = 0.5 * qw[i];
    /* eq. (qd4): w' = I^-1 (-w x (I w) + tau), I diagonal */
    const T Iw[3] = {t.Ixx * x[W + 0], t.Iyy * x[W + 1], t.Izz * x[W + 2]};
    const T wxIw[3] = {x[W + 1] * Iw[2] - x[W + 2] * Iw[1],
                       x[W + 2] * Iw[0] - x[W + 0] * Iw[2],
                       x[W + 0] * Iw[1] - x[W + 1] * Iw[0]};
    dx[W + 0] = (tau[0] - wxIw[0]) / t.Ixx;
    dx[W + 1] = (tau[1] - wxIw[1]) / t.Iyy;
    dx[W + 2] = (tau[2] - wxIw[2]) / t.Izz;
    /* first-order rotor lag toward the held command */
    for (int i = 0; i < 4; ++i) dx[M + i] = (Wcmd[i] - x[M + i]) / t.tau_m;
    /* running cost: sum of squared rotor speeds */
    dx[JC] = w2[0] + w2[1] + w2[2] + w2[3];
}

/* ------------------------------------------------------------------ */
/* Controller: position -> attitude -> body-rate PID cascade + mixer     */
/* ------------------------------------------------------------------ */

/* Evaluated once per step from the step-start state and held through all
 * four RK4 stages.  gains = [kpp kip kdp kpa kia kda kpr kir kdr]. */
template <class T>
void controller(const TypeData& td, const oracle_globals& gl, const T gains[9],
                const T x[NX], T mem[NMEM], const double wp[3], double dt, T Wcmd[4]) {
    const oracle_type& t = td.t;
    const T &kpp = gains[0], &kip = gains[1], &kdp = gains[2];
    const T &kpa = gains[3], &kia = gains[4], &kda = gains[5];
    const T &kpr = gains[6], &kir = gains[7], &kdr = gains[8];

    /* position loop: saturated error, clamped integral, D on velocity */
    T e[3];
    for (int i = 0; i < 3; ++i) e[i] = wp[i] - x[P + i];
    const T enorm = sqrt_(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    if (val(enorm) > gl.r_sat) {
        const T s = gl.r_sat / enorm;
        for (int i = 0; i < 3; ++i) e[i] = e[i] * s;
    }
    T a[3];
    for (int i = 0; i < 3; ++i) {
        mem[IP + i] = clamp_(mem[IP + i] + e[i] * dt, -gl.ipos_max, gl.ipos_max);
        a[i] = kpp * e[i] + kip * mem[IP + i] - kdp * x[V + i];
    }
    /* gravity feed-forward, keep the commanded vertical acceleration up */
    a[2] = a[2] + gl.g;
    if (val(a[2]) < gl.az_min_frac * gl.g) a[2] = T(gl.az_min_frac * gl.g);

    /* collective thrust: commanded acceleration projected on body z */
    T bz[3];
    body_z_axis(&x[Q], bz);
    const T fc = t.mass * (a[0] * bz[0] + a[1] * bz[1] + a[2] * bz[2]);

    /* desired attitude: smallest rotation taking z onto the thrust direction */
    const T anorm = sqrt_(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    const T n[3] = {a[0] / anorm, a[1] / anorm, a[2] / anorm};
    T qd[4] = {1.0 + n[2], -n[1], n[0], T(0.0)};
    const T qdn = sqrt_(qd[0] * qd[0] + qd[1] * qd[1] + qd[2] * qd[2] + qd[3] * qd[3]);
    for (int i = 0; i < 4; ++i) qd[i] = qd[i] / qdn;

    /* attitude loop: error quaternion conj(q) o q_des on the short arc */
    const T qc[4] = {x[Q + 0], -x[Q + 1], -x[Q + 2], -x[Q + 3]};
    T qe[4];
    quat_mul(qc, qd, qe);
    if (val(qe[0]) < 0.0)
        for (int i = 0; i < 4; ++i) qe[i] = -qe[i];
    T wdes[3];
    for (int i = 0; i < 3; ++i) {
        const T eatt = 2.0 * qe[1 + i];
        mem[IA + i] = clamp_(mem[IA + i] + eatt * dt, -gl.iatt_max, gl.iatt_max);
        wdes[i] = kpa * eatt + kia * mem[IA + i] - kda * x[W + i];
    }

    /* body-rate loop (the inner PID loop), D on measured rates */
    T alpha[3];
    for (int i = 0; i < 3; ++i) {
        const T ew = wdes[i] - x[W + i];
        mem[IR + i] = clamp_(mem[IR + i] + ew * dt, -gl.irate_max, gl.irate_max);
        alpha[i] = kpr * ew + kir * mem[IR + i] - kdr * (x[W + i] - mem[WPREV + i]) / dt;
    }
    for (int i = 0; i < 3; ++i) mem[WPREV + i] = x[W + i];

    /* desired torque: I alpha + w x (I w), inverse of eq. (qd4) */
    const T Iw[3] = {t.Ixx * x[W + 0], t.Iyy * x[W + 1], t.Izz * x[W + 2]};
    const T tau[3] = {t.Ixx * alpha[0] + (x[W + 1] * Iw[2] - x[W + 2] * Iw[1]),
                      t.Iyy * alpha[1] + (x[W + 2] * Iw[0] - x[W + 0] * Iw[2]),
                      t.Izz * alpha[2] + (x[W + 0] * Iw[1] - x[W + 1] * Iw[0])};

    /* mixer: solve eq. (3) for the rotor thrusts, saturate, invert eq. (2) */
    const T u[4] = {fc, tau[0], tau[1], tau[2]};
    const double fmax = t.k_f * t.w_max * t.w_max;
    for (int i = 0; i < 4; ++i) {
        T fi = td.Ginv[i][0] * u[0] + td.Ginv[i][1] * u[1] + td.Ginv[i][2] * u[2] + td.Ginv[i][3] * u[3];
        fi = clamp_(fi, 0.0, fmax);
        Wcmd[i] = sqrt_(fi / t.k_f);
    }
}

/* ------------------------------------------------------------------ */
/* One time step: controller (ZOH), classical RK4, renormalisation       */
/* ------------------------------------------------------------------ */

template <class T>
void rk4(const TypeData& td, double g, T x[NX], const T Wcmd[4], double h) {
    T k1[NX], k2[NX], k3[NX], k4[NX], xs[NX];
    derivative(td, g, x, Wcmd, k1);
    for (int i = 0; i < NX; ++i) xs[i] = x[i] + (0.5 * h) * k1[i];
    derivative(td, g, xs, Wcmd, k2);
    for (int i = 0; i < NX; ++i) xs[i] = x[i] + (0.5 * h) * k2[i];
    derivative(td, g, xs, Wcmd, k3);
    for (int i = 0; i < NX; ++i) xs[i] = x[i] + h * k3[i];
    derivative(td, g, xs, Wcmd, k4);
    for (int i = 0; i < NX; ++i)
        x[i] = x[i] + (h / 6.0) * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

template <class T>
void renormalise(T x[NX]) {
    const T n = sqrt_(x[Q] * x[Q] + x[Q + 1] * x[Q + 1] + x[Q + 2] * x[Q + 2] + x[Q + 3] * x[Q + 3]);
    for (int i = 0; i < 4; ++i) x[Q + i] = x[Q + i] / n;
}

struct Inputs {
    const TypeData* types;
    oracle_globals gl;
    int mode, renorm;
    const double* motor_cmd; int64_t cmd_ld;
    const double* wp; int n_epochs; int resample_every;
    int64_t step0; double dt;
};

/* Advance one agent `n` steps from global step index `step0`. */
template <class T>
void run_agent(const Inputs& in, const TypeData& td, const T gains[9], T x[NX], T mem[NMEM],
               int64_t agent, int64_t n) {
    double cmd[4] = {0, 0, 0, 0};
    if (in.mode == 0)
        for (int i = 0; i < 4; ++i) cmd[i] = td.t.w_ref + in.motor_cmd[i * in.cmd_ld + agent];
    for (int64_t k = 0; k < n; ++k) {
        T Wcmd[4];
        if (in.mode == 0) {
            for (int i = 0; i < 4; ++i) Wcmd[i] = T(cmd[i]);
        } else {
            int64_t ep = in.resample_every > 0 ? (in.step0 + k) / in.resample_every : 0;
            if (ep > in.n_epochs - 1) ep = in.n_epochs - 1;
            double wp[3];
            for (int i = 0; i < 3; ++i)
                wp[i] = in.wp[(ep * 3 + i) * in.cmd_ld + agent];
            controller(td, in.gl, gains, x, mem, wp, in.dt, Wcmd);
        }
        rk4(td, in.gl.g, x, Wcmd, in.dt);
        if (in.renorm) renormalise(x);
    }
}

int64_t steps_for(const oracle_type& t, int64_t step0, int64_t n_steps) {
    int64_t left = t.step_budget - step0;
    if (left < 0) left = 0;
    return left < n_steps ? left : n_steps;
}

}  // namespace

extern "C" {

/*
 * Advance n_agents agents n_steps steps in place.
 *   state     [30][ld] float64, row layout of the simulator (rotor rows hold
 *             the deviation from the type's w_ref, row 29 the running cost)
 *   type_idx  per-agent type (nullable: all type 0)
 *   gains     [9][gains_ld] per-agent gains (nullable: the type's gains)
 *   motor_cmd [4][cmd_ld] open-loop rotor commands (deviation from w_ref)
 *   wp        [n_epochs][3][cmd_ld] closed-loop waypoints
 * mode 0 = open loop (rows 0-16 touched), 1 = closed loop (all rows).
 * Returns 0, or -1 on invalid arguments / singular allocation matrix.
 */
int oracle_rollout(const oracle_type* types, int n_types, const oracle_globals* gl,
                   int mode, int renorm, double* state, int64_t ld, int64_t n_agents,
                   const int32_t* type_idx, const double* gains, int64_t gains_ld,
                   const double* motor_cmd, const double* wp, int n_epochs,
                   int resample_every, int64_t cmd_ld, int64_t step0, double dt,
                   int64_t n_steps, int n_threads) {
    if (!types || n_types < 1 || !gl || !state || ld < n_agents || n_agents < 0 || !(dt > 0.0))
        return -1;
    if (mode == 0 && !motor_cmd) return -1;
    if (mode == 1 && (!wp || n_epochs < 1)) return -1;
    TypeData td[256];
    if (n_types > 256) return -1;
    for (int t = 0; t < n_types; ++t)
        if (!make_type(types[t], td[t])) return -1;
    Inputs in{td, *gl, mode, renorm, motor_cmd, cmd_ld, wp, n_epochs, resample_every, step0, dt};
    if (n_threads < 1) n_threads = 1;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) num_threads(n_threads) reduction(| : bad)
    for (int64_t a = 0; a < n_agents; ++a) {
        const int ti = type_idx ? type_idx[a] : 0;
        if (ti < 0 || ti >= n_types) { bad = 1; continue; }
        const TypeData& T_ = td[ti];
        double x[NX], mem[NMEM], gn[9];
        for (int i = 0; i < 17; ++i) x[i] = state[i * ld + a];
        for (int i = 0; i < 4; ++i) x[M + i] += T_.t.w_ref;
        x[JC] = state[29 * ld + a];
        for (int i = 0; i < NMEM; ++i) mem[i] = state[(17 + i) * ld + a];
        for (int k = 0; k < 9; ++k) gn[k] = gains ? gains[k * gains_ld + a] : T_.t.gains[k];
        run_agent(in, T_, gn, x, mem, a, steps_for(T_.t, step0, n_steps));
        for (int i = 0; i < 4; ++i) x[M + i] -= T_.t.w_ref;
        for (int i = 0; i < 17; ++i) state[i * ld + a] = x[i];
        if (mode == 1) {
            for (int i = 0; i < NMEM; ++i) state[(17 + i) * ld + a] = mem[i];
            state[29 * ld + a] = x[JC];
        }
    }
    return bad ? -1 : 0;
}

/*
 * Jacobian of the closed-loop rollout map (x0[30], gains[9]) -> x_N[30] per
 * agent, by forward-mode dual numbers through the same templated step.
 * jac: [n_agents][30][39]; columns 0-29 initial-state rows, 30-38 gains.
 * The final state is written back to `state` as in oracle_rollout.
 */
int oracle_jacobian(const oracle_type* types, int n_types, const oracle_globals* gl,
                    double* state, int64_t ld, int64_t n_agents, const int32_t* type_idx,
                    const double* gains, int64_t gains_ld, const double* wp, int n_epochs,
                    int resample_every, int64_t cmd_ld, int64_t step0, double dt,
                    int64_t n_steps, double* jac, int n_threads) {
    typedef Dual<39> D;
    if (!types || n_types < 1 || n_types > 256 || !gl || !state || !jac || !wp || n_epochs < 1 ||
        ld < n_agents || n_agents < 0 || !(dt > 0.0))
        return -1;
    TypeData td[256];
    for (int t = 0; t < n_types; ++t)
        if (!make_type(types[t], td[t])) return -1;
    Inputs in{td, *gl, 1, 1, nullptr, cmd_ld, wp, n_epochs, resample_every, step0, dt};
    if (n_threads < 1) n_threads = 1;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads) reduction(| : bad)
    for (int64_t a = 0; a < n_agents; ++a) {
        const int ti = type_idx ? type_idx[a] : 0;
        if (ti < 0 || ti >= n_types) { bad = 1; continue; }
        const TypeData& T_ = td[ti];
        D x[NX], mem[NMEM], gn[9];
        for (int i = 0; i < 17; ++i) { x[i] = D(state[i * ld + a]); x[i].d[i] = 1.0; }
        for (int i = 0; i < 4; ++i) x[M + i].v += T_.t.w_ref;
        x[JC] = D(state[29 * ld + a]); x[JC].d[29] = 1.0;
        for (int i = 0; i < NMEM; ++i) { mem[i] = D(state[(17 + i) * ld + a]); mem[i].d[17 + i] = 1.0; }
        for (int k = 0; k < 9; ++k) {
            gn[k] = D(gains ? gains[k * gains_ld + a] : T_.t.gains[k]);
            gn[k].d[30 + k] = 1.0;
        }
        run_agent(in, T_, gn, x, mem, a, steps_for(T_.t, step0, n_steps));
        x[M + 0].v -= T_.t.w_ref; x[M + 1].v -= T_.t.w_ref;
        x[M + 2].v -= T_.t.w_ref; x[M + 3].v -= T_.t.w_ref;
        D out[30];
        for (int i = 0; i < 17; ++i) out[i] = x[i];
        for (int i = 0; i < NMEM; ++i) out[17 + i] = mem[i];
        out[29] = x[JC];
        for (int r = 0; r < 30; ++r) {
            state[r * ld + a] = out[r].v;
            for (int c = 0; c < 39; ++c) jac[(a * 30 + r) * 39 + c] = out[r].d[c];
        }
    }
    return bad ? -1 : 0;
}

/* Right-hand side f(x) for one agent: x[18] absolute rotor speeds, J last. */
int oracle_derivative(const oracle_type* type, double g, const double* x, const double* Wcmd,
                      double* dx) {
    TypeData td;
    if (!type || !make_type(*type, td)) return -1;
    derivative(td, g, x, Wcmd, dx);
    return 0;
}

/* One controller evaluation for one agent: x[18] (absolute rotor speeds),
 * mem[12] updated in place, returns absolute rotor commands Wcmd[4]. */
int oracle_controller(const oracle_type* type, const oracle_globals* gl, const double* gains,
                      const double* x, double* mem, const double* wp, double dt, double* Wcmd) {
    TypeData td;
    if (!type || !gl || !make_type(*type, td)) return -1;
    controller(td, *gl, gains ? gains : type->gains, x, mem, wp, dt, Wcmd);
    return 0;
}

/* The allocation matrix G of eq. (3) and its computed inverse. */
int oracle_allocation(const oracle_type* type, double* G, double* Ginv) {
    TypeData td;
    if (!type || !make_type(*type, td)) return -1;
    std::memcpy(G, td.G, sizeof(td.G));
    std::memcpy(Ginv, td.Ginv, sizeof(td.Ginv));
    return 0;
}

/*
 * Floating-point operations of one agent-step, by part of the step, counted
 * by the operation-counting scalar above (forward rules and reverse-sweep
 * rules are stated there).  counts[part * 6 + k], part 0 controller, 1 one
 * evaluation of the right-hand side f(x) (a step evaluates it four times),
 * 2 the RK4 stage and combination arithmetic outside f, 3 the quaternion
 * renormalisation; k = add/sub, mul, div, sqrt, comparisons, and the flops
 * of that part's reverse sweep.  mode 0 (open loop) has no controller part.
 * Evaluated at a generic flight state where no branch sits on a limit and
 * no input is exactly 0 or +-1.
 */
int oracle_count_ops(const oracle_type* type, const oracle_globals* gl, int mode, double dt,
                     int64_t* counts) {
    TypeData td;
    if (!type || !gl || !counts || !make_type(*type, td)) return -1;
    Cnt x[NX], mem[NMEM], gn[9];
    const double xs[NX] = {1.0, 2.0, 3.0, 0.1, -0.2, 0.05, 0.9995, 0.01, -0.02, 0.015,
                           0.03, -0.02, 0.01, 0, 0, 0, 0, 0.5};
    for (int i = 0; i < NX; ++i) x[i] = Cnt::input(xs[i]);
    for (int i = 0; i < 4; ++i) x[M + i] = Cnt::input(type->w_ref + 10.0 * (i - 1.5));
    /* integrals well inside their clamps; previous body rates close to the
     * current ones, so the commanded rotor thrusts stay inside [0, f_max] */
    for (int i = 0; i < 9; ++i) mem[i] = Cnt::input(0.01 * (i + 1));
    for (int i = 0; i < 3; ++i) mem[WPREV + i] = Cnt::input(xs[W + i] + 1e-4 * (i + 1));
    for (int k = 0; k < 9; ++k) gn[k] = Cnt::input(type->gains[k]);
    const double wp[3] = {1.5, 2.5, 3.2};
    auto take = [&](int part) {
        const int64_t v[6] = {g_ops.add, g_ops.mul, g_ops.div, g_ops.sqrt, g_ops.cmp, g_ops.rev};
        for (int k = 0; k < 6; ++k) counts[part * 6 + k] = v[k];
        std::memset(&g_ops, 0, sizeof(g_ops));
    };
    std::memset(counts, 0, sizeof(int64_t) * 24);
    std::memset(&g_ops, 0, sizeof(g_ops));
    Cnt Wcmd[4];
    if (mode == 1) {
        controller(td, *gl, gn, x, mem, wp, dt, Wcmd);
        take(0);
    } else {
        for (int i = 0; i < 4; ++i) Wcmd[i] = Cnt::input(type->w_ref * (1.0 + 0.01 * (i + 1)));
    }
    /* one right-hand side alone, then the whole RK4 step less four of them */
    Cnt dx[NX];
    derivative(td, gl->g, x, Wcmd, dx);
    take(1);
    rk4(td, gl->g, x, Wcmd, dt);
    const OpCount step = g_ops;
    std::memset(&g_ops, 0, sizeof(g_ops));
    const int64_t whole[6] = {step.add, step.mul, step.div, step.sqrt, step.cmp, step.rev};
    for (int k = 0; k < 6; ++k) counts[2 * 6 + k] = whole[k] - 4 * counts[1 * 6 + k];
    renormalise(x);
    take(3);
    return 0;
}

/*
 * Collision detection of Sec. II-A: agents closer than the sum of their
 * collision radii are marked dead (alive = 0) and excluded from then on.
 * All pairs of agents alive on entry are tested, brute force; the decisions
 * of one call are simultaneous (a pair kills both, a dead agent kills
 * nobody).  The decision |p_i - p_j|^2 < (r_i + r_j)^2 is taken in FP32 with
 * the operation order d2 = (dx*dx + dy*dy) + dz*dz, dx = x_i - x_j,
 * rr = (r_i + r_j) * (r_i + r_j), every operation rounded to float and no
 * fused multiply-add (this file is compiled without contraction).
 * rows: FP32 state rows [>=3][ld] (rows 0-2 are the position).
 * Returns the number of agents that died in this call, or -1 on bad input.
 */
int64_t oracle_detect_collisions(const float* rows, int64_t ld, int64_t n, const int32_t* type_idx,
                                 const float* radius, int n_types, uint8_t* alive) {
    if (!rows || !radius || !alive || n < 0 || ld < n || n_types < 1) return -1;
    const float* x = rows;
    const float* y = rows + ld;
    const float* z = rows + 2 * ld;
    uint8_t* hit = new uint8_t[n > 0 ? n : 1];
    for (int64_t i = 0; i < n; ++i) hit[i] = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!alive[i]) continue;
        const float ri = radius[type_idx ? type_idx[i] : 0];
        for (int64_t j = i + 1; j < n; ++j) {
            if (!alive[j]) continue;
            const float rj = radius[type_idx ? type_idx[j] : 0];
            const float dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            const float dxx = dx * dx, dyy = dy * dy, dzz = dz * dz;
            const float d2 = (dxx + dyy) + dzz;
            const float rs = ri + rj;
            const float rr = rs * rs;
            if (d2 < rr) { hit[i] = 1; hit[j] = 1; }
        }
    }
    int64_t died = 0;
    for (int64_t i = 0; i < n; ++i)
        if (hit[i]) { alive[i] = 0; ++died; }
    delete[] hit;
    return died;
}

/* The same decision for selected agents only: hit[q] = 1 when agent
 * query[q] (alive) collides with any other alive agent.  O(n) per query. */
int oracle_collides(const float* rows, int64_t ld, int64_t n, const int32_t* type_idx, const float* radius,
                    int n_types, const uint8_t* alive, const int64_t* query, int64_t n_query, uint8_t* hit,
                    int n_threads) {
    if (!rows || !radius || !alive || !query || !hit || n < 0 || ld < n || n_types < 1) return -1;
    const float* x = rows;
    const float* y = rows + ld;
    const float* z = rows + 2 * ld;
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
    for (int64_t q = 0; q < n_query; ++q) {
        const int64_t i = query[q];
        hit[q] = 0;
        if (i < 0 || i >= n || !alive[i]) continue;
        const float ri = radius[type_idx ? type_idx[i] : 0];
        for (int64_t j = 0; j < n; ++j) {
            if (j == i || !alive[j]) continue;
            const float rj = radius[type_idx ? type_idx[j] : 0];
            const float dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            const float dxx = dx * dx, dyy = dy * dy, dzz = dz * dz;
            const float d2 = (dxx + dyy) + dzz;
            const float rs = ri + rj;
            if (d2 < rs * rs) { hit[q] = 1; break; }
        }
    }
    return 0;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
