/*
 * vehicles.cpp -- plain FP64 CPU reference of the two other vehicle kinds
 * the simulator steps beside its quadrotors: a car and a fixed-wing
 * aircraft.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing but the test-suite, the smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no
 * source, header, constant or helper with the HIP kernels.
 *
 * The paper names three kinds of robot (fixed-wing drones, quadrotors and
 * cars, Sec. II-B, first paragraph) and writes out only the quadrotor; the
 * other two models are those of the works it cites for them, taken here as:
 *   - car: the kinematic bicycle model referenced at the centre of mass
 *     (Rajamani, "Vehicle Dynamics and Control", 2nd ed., 2012, Sec. 2.2),
 *     i.e. the dynamic bicycle model of the cited car work (Kabzan et al.,
 *     2019) without tyre slip; side-slip angle beta = atan(l_r tan(delta)/L),
 *     yaw rate v cos(beta) tan(delta)/L, a first-order steering actuator and
 *     a longitudinal acceleration input with linear drag;
 *   - fixed-wing: the kinematic guidance model of Beard and McLain ("Small
 *     Unmanned Aircraft", 2012, Ch. 9) in still air: ground speed along the
 *     course chi and flight-path angle gamma, the coordinated-turn course
 *     rate g tan(phi)/V, and first-order responses of the autopilot's
 *     airspeed, roll and flight-path loops;
 *   - guidance for both (closed loop): the orbit-following vector field of
 *     the same book (Ch. 10): fly a circle of radius rho around the
 *     waypoint, counter-clockwise for lambda = +1, clockwise for -1, with a
 *     course command that relaxes the radial error through
 *     atan(k_orb (d - rho)/rho), a steering or bank feed-forward that holds
 *     the circle exactly, and (fixed wing) a saturated altitude hold.  This
 *     gives the circle trajectories of the paper's first demo (Sec. IV).
 * Angles are in radians, counter-clockwise seen from above (ENU frame,
 * x east, y north, z up): heading and course measured from +x, positive
 * steering and positive bank both turn left.
 *
 * State rows used ([30][ld] layout of the simulator; others untouched):
 *   car:        0-2 position, 3 speed v, 4 yaw psi, 5 steering angle delta
 *   fixed-wing: 0-2 position, 3 airspeed V, 4 course chi, 5 bank phi,
 *               6 flight-path angle gamma
 * Open-loop commands ([4][cmd_ld], held for the whole call):
 *   car: 0 acceleration a_c, 1 steering command delta_c
 *   fixed-wing: 0 airspeed V_c, 1 bank phi_c, 2 flight-path gamma_c
 *
 * Pins (tests/test_vehicle_oracle.py): constant-steering and constant-bank
 * circles of closed-form radius, the straight run with drag and the
 * actuator lags in closed form, the steady helix, RK4's fourth order, the
 * orbit as an exact equilibrium of the guided closed loop, attraction to
 * the orbit, and mirror symmetry in lambda.  Parity unpinned: the guidance
 * gains and the feed-forward terms are this project's reading (the cited
 * works give the structure, not the numbers).
 */
#include <cmath>
#include <cstdint>
#include <omp.h>

extern "C" {

/* One vehicle type, FP64.  Field order is part of the ctypes binding.
 * veh[] by kind:
 *   car (kind 1):   0 L (wheelbase), 1 l_r (centre of mass to rear axle),
 *                   2 tau_delta, 3 delta_max, 4 a_max, 5 v_cruise, 6 rho,
 *                   7 lambda, 8 k_orb, 9 k_head, 10 k_speed
 *   fixed wing (2): 0 tau_V, 1 tau_phi, 2 tau_gamma, 3 phi_max, 4 gamma_max,
 *                   5 V_cruise, 6 rho, 7 lambda, 8 k_orb, 9 k_head, 10 k_alt */
typedef struct {
    int64_t kind;
    double mass, drag;
    double veh[12];
    int64_t step_budget;
} oracle_vehicle;

}  // extern "C"

namespace {

enum { KIND_CAR = 1, KIND_WING = 2 };
enum { PX = 0, PY = 1, PZ = 2, SPD = 3, HDG = 4, ACT = 5, FPA = 6, NV = 7 };

const double kPi = 3.14159265358979323846;

/* Angle a moved into [-pi, pi] by whole turns. */
double wrap_angle(double a) { return a - 2.0 * kPi * std::nearbyint(a / (2.0 * kPi)); }

double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

/* Car: kinematic bicycle at the centre of mass, inputs u = (a_c, delta_c). */
void car_rhs(const oracle_vehicle& t, const double x[NV], const double u[3], double dx[NV]) {
    const double L = t.veh[0], lr = t.veh[1], tau = t.veh[2];
    const double tan_d = std::tan(x[ACT]);
    const double beta = std::atan(lr * tan_d / L);
    dx[PX] = x[SPD] * std::cos(x[HDG] + beta);
    dx[PY] = x[SPD] * std::sin(x[HDG] + beta);
    dx[PZ] = 0.0;
    dx[SPD] = u[0] - (t.drag / t.mass) * x[SPD];
    dx[HDG] = x[SPD] * std::cos(beta) * tan_d / L;
    dx[ACT] = (u[1] - x[ACT]) / tau;
    dx[FPA] = 0.0;
}

/* Fixed wing: kinematic guidance model, inputs u = (V_c, phi_c, gamma_c). */
void wing_rhs(const oracle_vehicle& t, double g, const double x[NV], const double u[3], double dx[NV]) {
    const double V = x[SPD], chi = x[HDG], phi = x[ACT], gam = x[FPA];
    dx[PX] = V * std::cos(gam) * std::cos(chi);
    dx[PY] = V * std::cos(gam) * std::sin(chi);
    dx[PZ] = V * std::sin(gam);
    dx[SPD] = (u[0] - V) / t.veh[0];
    dx[HDG] = g * std::tan(phi) / V;
    dx[ACT] = (u[1] - phi) / t.veh[1];
    dx[FPA] = (u[2] - gam) / t.veh[2];
}

void rhs(const oracle_vehicle& t, double g, const double x[NV], const double u[3], double dx[NV]) {
    if (t.kind == KIND_CAR)
        car_rhs(t, x, u, dx);
    else
        wing_rhs(t, g, x, u, dx);
}

/* Course commanded by the orbit vector field around centre (cx, cy). */
double orbit_course(const oracle_vehicle& t, double x, double y, double cx, double cy) {
    const double rho = t.veh[6], lam = t.veh[7], k = t.veh[8];
    const double ex = x - cx, ey = y - cy;
    const double d = std::sqrt(ex * ex + ey * ey);
    const double around = std::atan2(ey, ex);
    return around + lam * (0.5 * kPi + std::atan(k * (d - rho) / rho));
}

/* Closed-loop inputs from the step-start state, held through the step. */
void guidance(const oracle_vehicle& t, double g, const double x[NV], const double wp[3], double u[3]) {
    const double chi_d = orbit_course(t, x[PX], x[PY], wp[0], wp[1]);
    const double rho = t.veh[6], lam = t.veh[7], k_head = t.veh[9];
    if (t.kind == KIND_CAR) {
        const double L = t.veh[0], lr = t.veh[1];
        /* the car's course is its yaw plus the side-slip angle */
        const double beta = std::atan(lr * std::tan(x[ACT]) / L);
        const double e = wrap_angle(chi_d - (x[HDG] + beta));
        /* steering that holds a circle of radius rho: rho^2 = L^2/tan^2 + l_r^2 */
        const double ff = lam * std::atan(L / std::sqrt(rho * rho - lr * lr));
        u[0] = clampd(t.veh[10] * (t.veh[5] - x[SPD]) + (t.drag / t.mass) * x[SPD], -t.veh[4], t.veh[4]);
        u[1] = clampd(ff + k_head * e, -t.veh[3], t.veh[3]);
        u[2] = 0.0;
    } else {
        const double e = wrap_angle(chi_d - x[HDG]);
        /* bank that holds a circle of radius rho: tan(phi) = V^2 / (g rho) */
        const double ff = lam * std::atan(x[SPD] * x[SPD] / (g * rho));
        u[0] = t.veh[5];
        u[1] = clampd(ff + k_head * e, -t.veh[3], t.veh[3]);
        u[2] = clampd(t.veh[10] * (wp[2] - x[PZ]), -t.veh[4], t.veh[4]);
    }
}

/* Classical RK4 with the inputs held. */
void rk4(const oracle_vehicle& t, double g, double x[NV], const double u[3], double h) {
    double k1[NV], k2[NV], k3[NV], k4[NV], xs[NV];
    rhs(t, g, x, u, k1);
    for (int i = 0; i < NV; ++i) xs[i] = x[i] + (0.5 * h) * k1[i];
    rhs(t, g, xs, u, k2);
    for (int i = 0; i < NV; ++i) xs[i] = x[i] + (0.5 * h) * k2[i];
    rhs(t, g, xs, u, k3);
    for (int i = 0; i < NV; ++i) xs[i] = x[i] + h * k3[i];
    rhs(t, g, xs, u, k4);
    for (int i = 0; i < NV; ++i) x[i] = x[i] + (h / 6.0) * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

bool valid(const oracle_vehicle& t) {
    if (t.kind != KIND_CAR && t.kind != KIND_WING) return false;
    if (!(t.mass > 0.0) || !(t.veh[6] > 0.0)) return false;
    if (t.kind == KIND_CAR) return t.veh[0] > 0.0 && t.veh[2] > 0.0 && t.veh[6] > t.veh[1];
    return t.veh[0] > 0.0 && t.veh[1] > 0.0 && t.veh[2] > 0.0;
}

}  // namespace

extern "C" {

/*
 * Advance n_agents vehicles n_steps steps in place (rows of the table at
 * the top of this file).  type_idx (nullable: all type 0) indexes `types`;
 * mode 0 holds motor_cmd [4][cmd_ld], mode 1 runs the orbit guidance around
 * wp[epoch][3][cmd_ld], epoch = min((step0 + k) / resample_every,
 * n_epochs - 1) (resample_every <= 0: epoch 0).  An agent takes
 * min(n_steps, max(0, step_budget - step0)) steps.  Returns 0, or -1 on
 * invalid arguments.
 */
int oracle_vehicle_rollout(const oracle_vehicle* types, int n_types, double g, int mode, double* state,
                           int64_t ld, int64_t n_agents, const int32_t* type_idx, const double* motor_cmd,
                           const double* wp, int n_epochs, int resample_every, int64_t cmd_ld, int64_t step0,
                           double dt, int64_t n_steps, int n_threads) {
    if (!types || n_types < 1 || n_types > 256 || !state || ld < n_agents || n_agents < 0 || !(dt > 0.0))
        return -1;
    if (mode == 0 && !motor_cmd) return -1;
    if (mode == 1 && (!wp || n_epochs < 1)) return -1;
    for (int t = 0; t < n_types; ++t)
        if (!valid(types[t])) return -1;
    if (n_threads < 1) n_threads = 1;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) num_threads(n_threads) reduction(| : bad)
    for (int64_t a = 0; a < n_agents; ++a) {
        const int ti = type_idx ? type_idx[a] : 0;
        if (ti < 0 || ti >= n_types) { bad = 1; continue; }
        const oracle_vehicle& t = types[ti];
        const int rows = t.kind == KIND_CAR ? 6 : 7;
        double x[NV] = {0, 0, 0, 0, 0, 0, 0};
        for (int i = 0; i < rows; ++i) x[i] = state[i * ld + a];
        int64_t left = t.step_budget - step0;
        if (left < 0) left = 0;
        const int64_t n = left < n_steps ? left : n_steps;
        double u[3] = {0, 0, 0};
        if (mode == 0)
            for (int i = 0; i < 3; ++i) u[i] = motor_cmd[i * cmd_ld + a];
        for (int64_t k = 0; k < n; ++k) {
            if (mode == 1) {
                int64_t ep = resample_every > 0 ? (step0 + k) / resample_every : 0;
                if (ep > n_epochs - 1) ep = n_epochs - 1;
                const double w[3] = {wp[(ep * 3 + 0) * cmd_ld + a], wp[(ep * 3 + 1) * cmd_ld + a],
                                     wp[(ep * 3 + 2) * cmd_ld + a]};
                guidance(t, g, x, w, u);
            }
            rk4(t, g, x, u, dt);
        }
        for (int i = 0; i < rows; ++i) state[i * ld + a] = x[i];
    }
    return bad ? -1 : 0;
}

/* Right-hand side of one vehicle: x[7] in the row order above, u[3]. */
int oracle_vehicle_derivative(const oracle_vehicle* type, double g, const double* x, const double* u, double* dx) {
    if (!type || !valid(*type)) return -1;
    rhs(*type, g, x, u, dx);
    return 0;
}

/* Closed-loop inputs of one vehicle at state x[7] and waypoint wp[3]. */
int oracle_vehicle_guidance(const oracle_vehicle* type, double g, const double* x, const double* wp, double* u) {
    if (!type || !valid(*type)) return -1;
    guidance(*type, g, x, wp, u);
    return 0;
}

}  // extern "C"
