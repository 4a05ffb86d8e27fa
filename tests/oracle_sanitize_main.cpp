/*
 * Driver for a host AddressSanitizer + UndefinedBehaviorSanitizer build of
 * the FP64 reference (test infrastructure: built and run by
 * tests/test_oracle_sanitizers.py with g++, never on a GPU).  It includes the
 * reference's source and calls each entry point on small inputs, including
 * ragged leading dimensions, per-agent gains and types, waypoint epochs and
 * the argument checks, so that out-of-bounds indexing or undefined
 * arithmetic in any of them aborts the run.
 */
#include "../oracle/oracle.cpp"

#include <cstdio>
#include <vector>

namespace {

oracle_type base_type(double scale) {
    oracle_type t{};
    t.mass = 1.0 * scale;
    t.Ixx = 0.0082 * scale; t.Iyy = 0.0082 * scale; t.Izz = 0.0149 * scale;
    t.arm = 0.17; t.alpha = 0.78539816339744831; t.k_f = 6.1e-6 * scale; t.k_m = 1.5e-7 * scale;
    t.tau_m = 0.02; t.drag = 0.1; t.w_max = 2500.0;
    t.w_ref = std::sqrt(t.mass * 9.81 / (4.0 * t.k_f));
    const double g[9] = {2, 0.1, 2, 8, 0.2, 0.1, 25, 2, 0.02};
    for (int k = 0; k < 9; ++k) t.gains[k] = g[k];
    t.step_budget = 1 << 30;
    return t;
}

int fail(const char* what) {
    std::fprintf(stderr, "FAILED: %s\n", what);
    return 1;
}

}  // namespace

int main() {
    const oracle_type types[2] = {base_type(1.0), base_type(1.7)};
    oracle_type budgeted[2] = {types[0], types[1]};
    budgeted[1].step_budget = 7;
    const oracle_globals gl{9.81, 2.0, 5.0, 1.0, 1.0, 0.5};
    const int64_t n = 5, ld = 7;           /* ragged: columns 5, 6 are padding */
    const int64_t steps = 23;
    std::vector<double> state(40 * ld, 0.0);
    for (int64_t a = 0; a < n; ++a) {
        state[0 * ld + a] = 1.0 + a;
        state[1 * ld + a] = -2.0 + 0.5 * a;
        state[2 * ld + a] = 3.0;
        state[6 * ld + a] = 1.0;
        for (int r = 13; r < 17; ++r) state[r * ld + a] = types[a & 1].w_ref;
    }
    const int32_t type_idx[5] = {0, 1, 0, 1, 1};
    std::vector<double> gains(9 * ld, 0.0);
    for (int k = 0; k < 9; ++k)
        for (int64_t a = 0; a < n; ++a) gains[k * ld + a] = types[0].gains[k] * (1.0 + 0.01 * a);
    const int n_epochs = 3;
    std::vector<double> wp(n_epochs * 3 * ld, 0.0);
    for (int e = 0; e < n_epochs; ++e)
        for (int r = 0; r < 3; ++r)
            for (int64_t a = 0; a < n; ++a) wp[(e * 3 + r) * ld + a] = 0.5 * (e + 1) + r - 0.1 * a;
    std::vector<double> cmd(4 * ld, 0.0);
    for (int r = 0; r < 4; ++r)
        for (int64_t a = 0; a < n; ++a) cmd[r * ld + a] = types[a & 1].w_ref * (1.0 + 0.01 * (r - a));

    /* closed loop, per-agent types, budgets, gains and waypoint epochs, 2 threads */
    std::vector<double> s = state;
    if (oracle_rollout(budgeted, 2, &gl, 1, 1, s.data(), ld, n, type_idx, gains.data(), ld, nullptr, wp.data(),
                       n_epochs, 8, ld, 3, 1e-3, steps, 2) != 0)
        return fail("closed-loop rollout");
    /* open loop, one type */
    s = state;
    if (oracle_rollout(types, 1, &gl, 0, 1, s.data(), ld, n, nullptr, nullptr, ld, cmd.data(), nullptr, 0, 0, ld, 0,
                       1e-3, steps, 1) != 0)
        return fail("open-loop rollout");
    /* argument checks */
    if (oracle_rollout(types, 1, &gl, 1, 1, s.data(), 3, n, nullptr, nullptr, ld, nullptr, wp.data(), 1, 0, ld, 0,
                       1e-3, steps, 1) == 0)
        return fail("ld < n accepted");
    /* dual-number Jacobian */
    s = state;
    std::vector<double> jac(n * 30 * 39, 0.0);
    if (oracle_jacobian(types, 2, &gl, s.data(), ld, n, type_idx, gains.data(), ld, wp.data(), n_epochs, 8, ld, 0,
                        2e-3, 11, jac.data(), 2) != 0)
        return fail("jacobian");
    /* single evaluations */
    double x[18] = {0}, dx[18] = {0}, wc[4];
    x[6] = 1.0;
    for (int i = 0; i < 4; ++i) { x[13 + i] = types[0].w_ref; wc[i] = types[0].w_ref * 1.05; }
    if (oracle_derivative(&types[0], 9.81, x, wc, dx) != 0) return fail("derivative");
    double mem[12] = {0}, out[4] = {0};
    const double target[3] = {1.0, 2.0, 3.0};
    if (oracle_controller(&types[0], &gl, nullptr, x, mem, target, 1e-3, out) != 0) return fail("controller");
    double G[16], Gi[16];
    if (oracle_allocation(&types[1], G, Gi) != 0) return fail("allocation");
    int64_t counts[24] = {0};
    if (oracle_count_ops(&types[0], &gl, 1, 1e-3, counts) != 0) return fail("count_ops");
    /* collisions: a pair inside the radius sum, a dead agent, a ragged ld */
    std::vector<float> rows(3 * ld, 0.0f);
    const float px[5] = {0.0f, 0.2f, 5.0f, 9.0f, 9.05f};
    for (int64_t a = 0; a < n; ++a) rows[a] = px[a];
    const float radius[2] = {0.17f, 0.05f};
    uint8_t alive[5] = {1, 1, 1, 1, 0};
    if (oracle_detect_collisions(rows.data(), ld, n, type_idx, radius, 2, alive) != 2) return fail("detect");
    const uint8_t alive2[5] = {1, 1, 1, 1, 1};
    const int64_t query[3] = {0, 3, 4};
    uint8_t hit[3] = {0, 0, 0};
    if (oracle_collides(rows.data(), ld, n, type_idx, radius, 2, alive2, query, 3, hit, 2) != 0)
        return fail("collides");
    if (!hit[0] || !hit[1] || !hit[2]) return fail("collides result");
    std::printf("oracle sanitizer run: ok\n");
    return 0;
}
