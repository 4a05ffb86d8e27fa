/*
 * Driver for a host AddressSanitizer + UndefinedBehaviorSanitizer build of
 * libpotato's host code (test infrastructure: built and run by
 * tests/test_abi_sanitizers.py, on a machine without a GPU or with one).
 * It calls every entry point along its argument-checking paths, which run
 * before any device work, and the context creation (which reaches the HIP
 * runtime), so that out-of-bounds accesses or undefined arithmetic in the
 * validation, constant derivation and error reporting abort the run.
 */
#include <cmath>
#include <cstdio>
#include <cstring>

#include "potato.h"

namespace {

int failures = 0;

void expect(bool ok, const char* what) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s (last error: %s)\n", what, potato_last_error(nullptr));
        ++failures;
    }
}

potato_type_params base_type() {
    potato_type_params t{};
    t.mass = 1.0f; t.Ixx = 0.0082f; t.Iyy = 0.0082f; t.Izz = 0.0149f; t.arm = 0.17f; t.alpha = 0.78539816f;
    t.k_f = 6.1e-6f; t.k_m = 1.5e-7f; t.tau_m = 0.02f; t.drag = 0.1f; t.w_max = 2500.0f; t.w_ref = 634.0f;
    t.radius = 0.17f;
    const float g[9] = {2, 0.1f, 2, 8, 0.2f, 0.1f, 25, 2, 0.02f};
    for (int k = 0; k < 9; ++k) t.gains[k] = g[k];
    t.step_budget = 1 << 30;
    return t;
}

}  // namespace

int main() {
    expect(std::strlen(potato_version()) > 0, "version");
    const potato_limits lim{9.81f, 2.0f, 5.0f, 1.0f, 1.0f, 0.5f};
    const potato_options opt{POTATO_CLOSED_LOOP, POTATO_FORM_FUSED, 0, 0, 0, 0};
    potato_type_params types[3] = {base_type(), base_type(), base_type()};
    potato_ctx* ctx = nullptr;

    /* context creation: every rejected argument, then a valid call */
    expect(potato_create(nullptr, types, 1, &lim, &opt) == POTATO_EINVAL, "create: null out");
    expect(potato_create(&ctx, nullptr, 1, &lim, &opt) == POTATO_EINVAL, "create: null types");
    expect(potato_create(&ctx, types, 0, &lim, &opt) == POTATO_EINVAL, "create: zero types");
    expect(potato_create(&ctx, types, POTATO_MAX_TYPES + 1, &lim, &opt) == POTATO_EINVAL, "create: too many types");
    types[1].mass = -1.0f;
    expect(potato_create(&ctx, types, 3, &lim, &opt) == POTATO_EINVAL, "create: negative mass");
    types[1] = base_type();
    types[2].alpha = 0.0f;
    expect(potato_create(&ctx, types, 3, &lim, &opt) == POTATO_EINVAL, "create: alpha 0");
    types[2] = base_type();
    types[0].gains[4] = NAN;
    expect(potato_create(&ctx, types, 3, &lim, &opt) == POTATO_EINVAL, "create: NaN gain");
    types[0] = base_type();
    potato_limits bad_lim = lim;
    bad_lim.r_sat = 0.0f;
    expect(potato_create(&ctx, types, 3, &bad_lim, &opt) == POTATO_EINVAL, "create: r_sat 0");
    potato_options bad_opt = opt;
    bad_opt.block = 100;
    expect(potato_create(&ctx, types, 3, &lim, &bad_opt) == POTATO_EINVAL, "create: block 100");
    bad_opt = opt;
    bad_opt.mode = 2;
    expect(potato_create(&ctx, types, 3, &lim, &bad_opt) == POTATO_EINVAL, "create: mode 2");
    const potato_status made = potato_create(&ctx, types, 3, &lim, &opt);
    expect(made == POTATO_OK || made == POTATO_EHIP, "create: valid arguments");
    expect(made == POTATO_OK ? ctx != nullptr : ctx == nullptr, "create: handle matches status");

    /* every other entry point on null handles */
    potato_state st{nullptr, 10, nullptr, 0};
    potato_params pp{};
    potato_cmds cm{};
    expect(potato_destroy(nullptr) == POTATO_OK, "destroy null");
    expect(potato_set_options(nullptr, &opt) == POTATO_EINVAL, "set_options null");
    expect(potato_step(nullptr, &st, &pp, &cm, 1e-3f, 10, 1, nullptr, 0, nullptr) == POTATO_EINVAL, "step null");
    expect(potato_autotune(nullptr, &st, &pp, &cm, 1e-3f, 10, 10, 0, nullptr, nullptr) == POTATO_EINVAL, "autotune null");
    expect(potato_order_workspace_bytes(0, 8) == -1 && potato_order_workspace_bytes(10, 0) == -1, "order workspace");
    expect(potato_order_workspace_bytes(1000, 8) > 0, "order workspace size");
    expect(potato_order_by_type(nullptr, nullptr, 10, nullptr, nullptr, 0, nullptr) == POTATO_EINVAL, "order null");
    expect(potato_backward_workspace_bytes(nullptr, &pp, 10, 5) == -1, "backward workspace null");
    expect(potato_step_backward(nullptr, &pp, &cm, 1e-3f, 10, 10, nullptr, 5, 10, nullptr, nullptr, nullptr,
                                nullptr, nullptr, 0, nullptr) == POTATO_EINVAL, "backward null");
    expect(potato_collision_workspace_bytes(0) == -1 && potato_collision_workspace_bytes(1000) > 0,
           "collision workspace");
    expect(potato_detect_collisions(nullptr, &st, &pp, 10, nullptr, nullptr, nullptr, 0, nullptr) == POTATO_EINVAL,
           "detect null");
    potato_pipe* pipe = nullptr;
    expect(potato_pipe_create(nullptr, 10, &pipe) == POTATO_EINVAL, "pipe create null ctx");
    expect(potato_pipe_push(nullptr, nullptr) == POTATO_EINVAL, "pipe push null");
    expect(potato_pipe_run(nullptr, &st, &pp, 1e-3f, 1, 0, nullptr, nullptr) == POTATO_EINVAL, "pipe run null");
    expect(potato_pipe_wait_snapshots(nullptr, 0) == POTATO_EINVAL, "pipe wait null");
    expect(potato_pipe_sync(nullptr) == POTATO_EINVAL, "pipe sync null");
    int64_t a = 0, b = 0;
    expect(potato_pipe_stats(nullptr, &a, &b) == POTATO_EINVAL, "pipe stats null");
    expect(potato_pipe_destroy(nullptr) == POTATO_OK, "pipe destroy null");
    expect(potato_count_nonfinite(nullptr, &st, 10, nullptr, nullptr) == POTATO_EINVAL, "count_nonfinite null");

    /* with a context (a GPU is present): argument errors of the calls */
    if (ctx) {
        expect(potato_step(ctx, &st, &pp, &cm, 1e-3f, 10, 1, nullptr, 0, nullptr) == POTATO_EINVAL,
               "step: null rows");
        expect(potato_step(ctx, &st, &pp, &cm, -1.0f, 10, 1, nullptr, 0, nullptr) == POTATO_EINVAL, "step: dt < 0");
        expect(potato_pipe_create(ctx, 0, &pipe) == POTATO_EINVAL, "pipe create: zero agents");
        expect(potato_destroy(ctx) == POTATO_OK, "destroy");
    }
    expect(std::strlen(potato_last_error(nullptr)) > 0, "last error kept");
    if (failures) return 1;
    std::printf("abi sanitizer run: ok\n");
    return 0;
}
