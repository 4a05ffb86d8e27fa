/*
 * abi.hip -- host side of the C ABI declared in include/potato.h: argument
 * validation, per-type constant derivation, launch policy (plain / fused,
 * autotuned block, steps per launch and grid), hipGraph capture and replay,
 * and the type-ordering helper for heterogeneous batches.
 */
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/potato.h"
#include "internal.h"
#include "kernels.h"

using namespace potato;

namespace {

thread_local std::string g_err;

potato_status fail(potato_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

potato_status hip_fail(hipError_t e, const char* where) {
    return fail(POTATO_EHIP, "%s: %s", where, hipGetErrorString(e));
}

bool finite_pos(float x) { return std::isfinite(x) && x > 0.0f; }

struct TuneKey {
    int mode, het, gains, perm, ckpt;
    bool operator<(const TuneKey& o) const {
        return std::tie(mode, het, gains, perm, ckpt) < std::tie(o.mode, o.het, o.gains, o.perm, o.ckpt);
    }
};
struct Tuned { int block, steps, grid; };

}  // namespace

struct potato_ctx {
    int device = 0;
    int n_types = 0;
    bool kinds = false;                /* some type is a car or fixed-wing aircraft */
    int n_groups = 0;                  /* classes grouped within a block (2..kMaxGroups), or 0 */
    std::vector<potato_type_params> params;
    std::vector<TypeConst> consts;
    TypeConst* d_table = nullptr;
    int32_t* d_rank = nullptr;         /* rank of each type by budget (longest first) */
    float* d_radius = nullptr;         /* collision radius per type */
    float r_max = 0.0f;
    void* scratch = nullptr;           /* this device's static collision workspace */
    int64_t scratch_bytes = 0;
    potato_limits limits{};
    potato_options opts{};
    hipStream_t cap_stream = nullptr;
    std::map<std::vector<int64_t>, hipGraphExec_t> graphs;
    std::map<TuneKey, Tuned> tuned;
    std::mutex mu;
};

namespace {

/* Per-type constants.  Derived once per context on the host in double and
 * rounded to FP32; every per-agent operation on the device is FP32. */
TypeConst derive(const potato_type_params& p, const potato_limits& L) {
    TypeConst c{};
    const double m = p.mass, kf = p.k_f, km = p.k_m, w = p.w_ref;
    const double ls = (double)p.arm * std::sin((double)p.alpha);
    const double lc = (double)p.arm * std::cos((double)p.alpha);
    const double F0 = 4.0 * kf * w * w / m;
    c.mass = p.mass;
    c.inv_m = (float)(1.0 / m);
    c.cd_m = (float)(p.drag / m);
    c.ncd_m = -c.cd_m;
    c.Ix = p.Ixx; c.Iy = p.Iyy; c.Iz = p.Izz;
    c.iIx = (float)(1.0 / p.Ixx); c.iIy = (float)(1.0 / p.Iyy); c.iIz = (float)(1.0 / p.Izz);
    c.F0 = (float)F0;
    c.F0_g = (float)(F0 - (double)L.g);
    c.kf_m = (float)(kf / m);
    c.F0_2 = 2.0f * c.F0;
    c.kf_m2 = 2.0f * c.kf_m;
    c.kf_ls = (float)(kf * ls);
    c.kf_lc = (float)(kf * lc);
    c.km = p.k_m;
    c.ax = (float)(kf * ls / p.Ixx);
    c.ay = (float)(kf * lc / p.Iyy);
    c.az = (float)(km / p.Izz);
    c.gx = (float)(((double)p.Izz - p.Iyy) / p.Ixx);
    c.gy = (float)(((double)p.Ixx - p.Izz) / p.Iyy);
    c.gz = (float)(((double)p.Iyy - p.Ixx) / p.Izz);
    c.w_ref = p.w_ref;
    c.two_w = (float)(2.0 * w);
    c.four_w2 = (float)(4.0 * w * w);
    c.inv_tau = (float)(1.0 / p.tau_m);
    c.mix_x = (float)(1.0 / (4.0 * ls));
    c.mix_y = (float)(1.0 / (4.0 * lc));
    c.mix_z = (float)(kf / (4.0 * km));
    c.f_max = (float)(kf * (double)p.w_max * (double)p.w_max);
    c.inv_kf = (float)(1.0 / kf);
    for (int k = 0; k < 9; ++k) c.gains[k] = p.gains[k];
    c.budget = p.step_budget;
    c.kind = KIND_QUAD;
    return c;
}

/* Constants of a car or fixed-wing type (kinds 1, 2), in double rounded to
 * FP32 like the quadrotor's. */
TypeConst derive_vehicle(const potato_type_params& p, const potato_limits& L) {
    TypeConst c{};
    VehConst& v = c.veh;
    double x[12];
    for (int k = 0; k < 12; ++k) x[k] = p.veh[k];
    const double pi = 3.14159265358979323846;
    v.rho = p.veh[6];
    v.lam = p.veh[7];
    v.lam_half_pi = (float)(x[7] * 0.5 * pi);
    v.k_orb_rho = (float)(x[8] / x[6]);
    v.k_head = p.veh[9];
    v.k_hold = p.veh[10];
    if (p.kind == POTATO_KIND_CAR) {
        const double Lw = x[0], lr = x[1];
        v.inv_tau[0] = (float)(1.0 / x[2]);
        v.lim[0] = p.veh[4];
        v.lim[1] = p.veh[3];
        v.cruise = p.veh[5];
        v.cd_m = (float)((double)p.drag / (double)p.mass);
        v.inv_L = (float)(1.0 / Lw);
        v.lr_L = (float)(lr / Lw);
        v.ff = (float)(x[7] * std::atan(Lw / std::sqrt(x[6] * x[6] - lr * lr)));
    } else {
        v.inv_tau[0] = (float)(1.0 / x[0]);
        v.inv_tau[1] = (float)(1.0 / x[1]);
        v.inv_tau[2] = (float)(1.0 / x[2]);
        v.lim[1] = p.veh[3];
        v.lim[2] = p.veh[4];
        v.cruise = p.veh[5];
        v.inv_g_rho = (float)(1.0 / ((double)L.g * x[6]));
        v.g = L.g;
    }
    c.budget = p.step_budget;
    c.kind = (int16_t)p.kind;
    return c;
}

Limits make_limits(const potato_limits& L, float dt) {
    Limits r{};
    r.g = L.g;
    r.r_sat = L.r_sat;
    r.r_sat2 = L.r_sat * L.r_sat;
    r.ipos_max = L.ipos_max;
    r.iatt_max = L.iatt_max;
    r.irate_max = L.irate_max;
    r.az_min = L.az_min_frac * L.g;
    r.dt = dt;
    r.half_dt = 0.5f * dt;
    r.dt6 = dt / 6.0f;
    r.quarter_dt = 0.5f * r.half_dt;
    r.dt12 = 0.5f * r.dt6;
    r.inv_dt = 1.0f / dt;
    r.dt2_6 = dt * dt / 6.0f;
    return r;
}

potato_status check_vehicle(const potato_type_params& p, int t) {
    if (!finite_pos(p.mass)) return fail(POTATO_EINVAL, "type %d: mass must be finite and > 0", t);
    if (!std::isfinite(p.drag) || p.drag < 0.0f || !std::isfinite(p.radius) || p.radius < 0.0f)
        return fail(POTATO_EINVAL, "type %d: drag and radius must be finite and >= 0", t);
    for (int k = 0; k < 12; ++k)
        if (!std::isfinite(p.veh[k])) return fail(POTATO_EINVAL, "type %d: veh[%d] must be finite", t, k);
    const float* v = p.veh;
    if (p.kind == POTATO_KIND_CAR) {
        if (!finite_pos(v[0]) || !finite_pos(v[2]) || !finite_pos(v[6]) || !(v[6] > v[1]) || v[1] < 0.0f)
            return fail(POTATO_EINVAL, "type %d (car): need L > 0, tau_delta > 0, 0 <= l_r < rho", t);
        if (v[3] < 0.0f || v[4] < 0.0f)
            return fail(POTATO_EINVAL, "type %d (car): delta_max and a_max must be >= 0", t);
    } else {
        if (!finite_pos(v[0]) || !finite_pos(v[1]) || !finite_pos(v[2]) || !finite_pos(v[5]) || !finite_pos(v[6]))
            return fail(POTATO_EINVAL, "type %d (fixed wing): need time constants, V_cruise and rho > 0", t);
        if (v[3] < 0.0f || v[4] < 0.0f)
            return fail(POTATO_EINVAL, "type %d (fixed wing): phi_max and gamma_max must be >= 0", t);
    }
    return POTATO_OK;
}

potato_status check_type(const potato_type_params& p, int t) {
    if (p.kind == POTATO_KIND_CAR || p.kind == POTATO_KIND_WING) return check_vehicle(p, t);
    if (p.kind != POTATO_KIND_QUAD) return fail(POTATO_EINVAL, "type %d: kind must be 0, 1 or 2", t);
    const float vals[] = {p.mass, p.Ixx, p.Iyy, p.Izz, p.arm, p.k_f, p.k_m, p.tau_m};
    for (float v : vals)
        if (!finite_pos(v)) return fail(POTATO_EINVAL, "type %d: mass, inertia, arm, k_f, k_m, tau_m must be finite and > 0", t);
    if (!std::isfinite(p.alpha) || std::fabs(std::sin(p.alpha)) < 1e-6f || std::fabs(std::cos(p.alpha)) < 1e-6f)
        return fail(POTATO_EINVAL, "type %d: alpha must be finite with sin and cos away from 0", t);
    if (!std::isfinite(p.drag) || p.drag < 0.0f || !std::isfinite(p.w_max) || p.w_max < 0.0f ||
        !std::isfinite(p.w_ref) || p.w_ref < 0.0f || !std::isfinite(p.radius) || p.radius < 0.0f)
        return fail(POTATO_EINVAL, "type %d: drag, w_max, w_ref, radius must be finite and >= 0", t);
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(p.gains[k])) return fail(POTATO_EINVAL, "type %d: gains must be finite", t);
    return POTATO_OK;
}

potato_status check_limits(const potato_limits& L) {
    if (!finite_pos(L.g) || !finite_pos(L.r_sat) || !std::isfinite(L.ipos_max) || L.ipos_max < 0 ||
        !std::isfinite(L.iatt_max) || L.iatt_max < 0 || !std::isfinite(L.irate_max) || L.irate_max < 0 ||
        !finite_pos(L.az_min_frac))
        return fail(POTATO_EINVAL, "limits: g, r_sat, az_min_frac must be > 0; integral clamps >= 0");
    return POTATO_OK;
}

potato_status check_options(const potato_options& o) {
    if (o.mode != POTATO_OPEN_LOOP && o.mode != POTATO_CLOSED_LOOP)
        return fail(POTATO_EINVAL, "options.mode must be 0 (open loop) or 1 (closed loop)");
    if (o.form < POTATO_FORM_AUTO || o.form > POTATO_FORM_FUSED)
        return fail(POTATO_EINVAL, "options.form must be 0, 1 or 2");
    if (!(o.block == 0 || o.block == 64 || o.block == 128 || o.block == 256 || o.block == 512 || o.block == 1024))
        return fail(POTATO_EINVAL, "options.block must be 0, 64, 128, 256, 512 or 1024");
    if (o.steps_per_launch < 0 || o.grid_blocks < 0)
        return fail(POTATO_EINVAL, "options.steps_per_launch and grid_blocks must be >= 0");
    return POTATO_OK;
}

void drop_graphs(potato_ctx* ctx) {
    for (auto& kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
    ctx->graphs.clear();
}

struct Plan {
    Variant v;
    StepArgs a;
    int block, steps, grid;
};

potato_status validate_step(const potato_ctx* ctx, const potato_state* st, const potato_params* pp,
                            const potato_cmds* cm, float dt, int64_t n, int32_t n_steps,
                            const float* ckpt, int32_t ckpt_every) {
    if (!ctx || !st || !pp || !cm) return fail(POTATO_EINVAL, "ctx, state, params and cmds must be non-null");
    if (!st->rows) return fail(POTATO_EINVAL, "state.rows is null");
    if (n < 1) return fail(POTATO_EINVAL, "n_agents must be >= 1");
    if (n > kMaxAgents) return fail(POTATO_EINVAL, "n_agents must be <= 2^30");
    if (st->ld < n) return fail(POTATO_EINVAL, "state.ld (%lld) < n_agents (%lld)", (long long)st->ld, (long long)n);
    if (st->carry && st->carry_ld < n)
        return fail(POTATO_EINVAL, "state.carry_ld (%lld) < n_agents (%lld)", (long long)st->carry_ld, (long long)n);
    if (n_steps < 0) return fail(POTATO_EINVAL, "n_steps must be >= 0");
    if (!std::isfinite(dt) || !(dt > 0.0f)) return fail(POTATO_EINVAL, "dt must be finite and > 0");
    if (cm->ld < n) return fail(POTATO_EINVAL, "cmds.ld < n_agents");
    if (cm->step0 < 0) return fail(POTATO_EINVAL, "cmds.step0 must be >= 0");
    if (ctx->opts.mode == POTATO_OPEN_LOOP) {
        if (!cm->motor_cmd) return fail(POTATO_EINVAL, "open loop needs cmds.motor_cmd");
        if (ckpt) return fail(POTATO_EUNSUPPORTED, "checkpoints are only produced in closed loop");
    } else {
        if (!cm->wp || cm->n_epochs < 1) return fail(POTATO_EINVAL, "closed loop needs cmds.wp and n_epochs >= 1");
    }
    if (pp->gains && pp->gains_ld < n) return fail(POTATO_EINVAL, "params.gains_ld < n_agents");
    if (ckpt && ckpt_every < 1) return fail(POTATO_EINVAL, "ckpt_every must be >= 1 when ckpt is given");
    if (ckpt && !st->carry)
        return fail(POTATO_EINVAL, "checkpoints need the rounding carries (state.carry): the adjoint replays the "
                                   "compensated integrator");
    if (ckpt && ctx->opts.form == POTATO_FORM_PLAIN)
        return fail(POTATO_EUNSUPPORTED, "checkpoints need the fused form");
    if (ckpt && ctx->kinds)
        return fail(POTATO_EUNSUPPORTED, "checkpoints (the adjoint) cover quadrotors only; the type table "
                                         "holds cars or fixed-wing aircraft");
    if (pp->type == nullptr && pp->perm != nullptr)
        return fail(POTATO_EUNSUPPORTED, "params.perm needs params.type");
    return POTATO_OK;
}

Plan make_plan(potato_ctx* ctx, const potato_state* st, const potato_params* pp, const potato_cmds* cm,
               float dt, int64_t n, float* ckpt, int32_t ckpt_every) {
    Plan P{};
    P.v.mode = ctx->opts.mode;
    P.v.het = pp->type != nullptr;
    P.v.gains = ctx->opts.mode == POTATO_CLOSED_LOOP && pp->gains != nullptr;
    P.v.ckpt = ckpt != nullptr;
    P.v.perm = P.v.het && pp->perm != nullptr;
    P.v.carry = st->carry != nullptr;
    /* a homogeneous launch stages type 0 only */
    P.v.kinds = P.v.het ? ctx->kinds : ctx->consts[0].kind != KIND_QUAD;
    StepArgs& a = P.a;
    a.rows = st->rows; a.ld = st->ld; a.n = n;
    a.carry = st->carry; a.carry_ld = st->carry ? st->carry_ld : 0;
    a.type = pp->type; a.perm = P.v.perm ? pp->perm : nullptr;
    a.gains = P.v.gains ? pp->gains : nullptr; a.gains_ld = pp->gains_ld;
    a.motor_cmd = cm->motor_cmd; a.wp = cm->wp; a.cmd_ld = cm->ld;
    a.n_epochs = cm->n_epochs < 1 ? 1 : cm->n_epochs; a.resample = cm->resample_every;
    a.step0 = cm->step0; a.k0 = 0; a.n_steps = 0;
    a.ckpt = ckpt; a.ckpt_every = ckpt_every > 0 ? ckpt_every : 1;
    a.n_types = ctx->n_types; a.table = ctx->d_table;
    a.alive = pp->alive;
    a.snap = nullptr;
    a.lim = make_limits(ctx->limits, dt);
    if (!P.v.het) a.n_types = 1;      /* homogeneous launch: only type 0 is staged */
    a.n_groups = P.v.het && !P.v.perm ? ctx->n_groups : 0;

    const potato_options& o = ctx->opts;
    /* agents grouped per block: the widest blocks measured best (mixed
     * kinds at 1M agents, 512 threads: 9.3e10 agent-steps/s against 8.2e10
     * with 256 and 7.0e10 with 128): more agents per block fill the groups
     * of rare classes, and more waves share out the groups more evenly */
    Tuned t{rollout_grouped(P.v, P.a) ? 1024 : 256, 100, 0};
    auto it = ctx->tuned.find(TuneKey{P.v.mode, P.v.het, P.v.gains, P.v.perm, P.v.ckpt});
    if (it != ctx->tuned.end()) t = it->second;
    if (o.form == POTATO_FORM_PLAIN) {
        /* one step per launch is HBM bound: 128-thread blocks measured best
         * (6.6 TB/s at 1M agents, against 6.2 with 256 and 5.2 with 512) */
        P.block = o.block ? o.block : 128;
        P.steps = 1;
        P.grid = 0;
    } else {
        P.block = o.block ? o.block : t.block;
        P.steps = o.steps_per_launch ? o.steps_per_launch : t.steps;
        P.grid = o.grid_blocks ? o.grid_blocks : t.grid;
    }
    return P;
}

/* `snap` (device view of mapped host memory, [3][n], or null) receives every
 * agent's position from the last launch. */
hipError_t enqueue(const Plan& P, int32_t n_steps, hipStream_t s, float* snap = nullptr) {
    StepArgs a = P.a;
    for (int32_t k0 = 0; k0 < n_steps; k0 += P.steps) {
        a.k0 = k0;
        a.step0 = P.a.step0 + k0;
        a.n_steps = std::min(P.steps, n_steps - k0);
        a.snap = k0 + a.n_steps == n_steps ? snap : nullptr;
        hipError_t e = launch_rollout(P.v, a, P.block, P.grid, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

std::vector<int64_t> graph_key(const Plan& P, int32_t n_steps, float dt) {
    const StepArgs& a = P.a;
    int32_t dtbits;
    std::memcpy(&dtbits, &dt, 4);
    return {(int64_t)a.rows, a.ld, a.n, (int64_t)a.type, (int64_t)a.perm, (int64_t)a.gains, a.gains_ld,
            (int64_t)a.motor_cmd, (int64_t)a.wp, a.cmd_ld, a.n_epochs, a.resample, a.step0, n_steps,
            dtbits, (int64_t)a.ckpt, a.ckpt_every, P.block, P.steps, P.grid, P.v.mode, (int64_t)a.alive,
            (int64_t)a.carry, a.carry_ld};
}

}  // namespace

namespace potato {

potato_status set_error(potato_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

potato_status set_hip_error(hipError_t e, const char* where) { return hip_fail(e, where); }

int ctx_mode(const potato_ctx* ctx) { return ctx->opts.mode; }

int ctx_device(const potato_ctx* ctx) { return ctx->device; }

potato_status step_eager(potato_ctx* ctx, const potato_state* state, const potato_params* params,
                         const potato_cmds* cmds, float dt, int64_t n_agents, int32_t n_steps,
                         hipStream_t stream, float* snap) {
    potato_status s = validate_step(ctx, state, params, cmds, dt, n_agents, n_steps, nullptr, 0);
    if (s != POTATO_OK) return s;
    if (n_steps == 0) return POTATO_OK;
    std::lock_guard<std::mutex> g(ctx->mu);
    Plan P = make_plan(ctx, state, params, cmds, dt, n_agents, nullptr, 0);
    hipError_t e = enqueue(P, n_steps, stream, snap);
    return e == hipSuccess ? POTATO_OK : hip_fail(e, "potato step launch");
}

}  // namespace potato

extern "C" {

potato_status potato_create(potato_ctx** out, const potato_type_params* types, int32_t n_types,
                            const potato_limits* limits, const potato_options* opts) {
    if (!out) return fail(POTATO_EINVAL, "out is null");
    *out = nullptr;
    if (!types || !limits || !opts) return fail(POTATO_EINVAL, "types, limits and opts must be non-null");
    if (n_types < 1 || n_types > POTATO_MAX_TYPES) return fail(POTATO_EINVAL, "n_types must be in [1, 256]");
    for (int t = 0; t < n_types; ++t) {
        potato_status s = check_type(types[t], t);
        if (s != POTATO_OK) return s;
    }
    potato_status s = check_limits(*limits);
    if (s != POTATO_OK) return s;
    s = check_options(*opts);
    if (s != POTATO_OK) return s;

    potato_ctx* ctx = new (std::nothrow) potato_ctx();
    if (!ctx) return fail(POTATO_ENOMEM, "host allocation failed");
    ctx->n_types = n_types;
    ctx->params.assign(types, types + n_types);
    ctx->limits = *limits;
    ctx->opts = *opts;
    for (int t = 0; t < n_types; ++t) {
        const bool quad = types[t].kind == POTATO_KIND_QUAD;
        ctx->consts.push_back(quad ? derive(types[t], *limits) : derive_vehicle(types[t], *limits));
        ctx->kinds = ctx->kinds || !quad;
    }
    /* classes of types that take the same steps of the same loop (equal
     * budget and kind), numbered longest first: by budget, then by the
     * kind's step (measured per agent-step at 1M agents, each kind alone in
     * the type order: fixed wing 11.0 ps, quadrotor 9.5, car 8.2).
     * Launches with a per-agent type and no processing order group their
     * agents by class within each block when there are 2..kMaxGroups
     * classes. */
    {
        auto cost = [](int32_t kind) { return kind == KIND_WING ? 2 : kind == KIND_QUAD ? 1 : 0; };
        std::vector<std::pair<int32_t, int>> cls;
        for (int t = 0; t < n_types; ++t) cls.emplace_back(ctx->consts[t].budget, cost(ctx->consts[t].kind));
        std::sort(cls.begin(), cls.end(), std::greater<std::pair<int32_t, int>>());
        cls.erase(std::unique(cls.begin(), cls.end()), cls.end());
        const bool group = cls.size() >= 2 && cls.size() <= (size_t)kMaxGroups;
        ctx->n_groups = group ? (int)cls.size() : 0;
        for (int t = 0; t < n_types; ++t) {
            const std::pair<int32_t, int> key(ctx->consts[t].budget, cost(ctx->consts[t].kind));
            ctx->consts[t].group =
                group ? (int16_t)(std::find(cls.begin(), cls.end(), key) - cls.begin()) : 0;
        }
    }
    /* rank of each type: longest budget first, ties by index */
    std::vector<int32_t> order(n_types), rank(n_types);
    for (int t = 0; t < n_types; ++t) order[t] = t;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return types[a].step_budget > types[b].step_budget; });
    for (int r = 0; r < n_types; ++r) rank[order[r]] = r;

    std::vector<float> radius(n_types);
    for (int t = 0; t < n_types; ++t) {
        radius[t] = types[t].radius;
        ctx->r_max = std::max(ctx->r_max, types[t].radius);
    }
    hipError_t e = hipGetDevice(&ctx->device);
    if (e == hipSuccess) e = hipMalloc(&ctx->d_table, sizeof(TypeConst) * n_types);
    if (e == hipSuccess) e = hipMalloc(&ctx->d_rank, sizeof(int32_t) * n_types);
    if (e == hipSuccess) e = hipMalloc(&ctx->d_radius, sizeof(float) * n_types);
    if (e == hipSuccess)
        e = hipMemcpy(ctx->d_radius, radius.data(), sizeof(float) * n_types, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(ctx->d_table, ctx->consts.data(), sizeof(TypeConst) * n_types, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->d_rank, rank.data(), sizeof(int32_t) * n_types, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = collision_scratch(&ctx->scratch, &ctx->scratch_bytes);
    if (e != hipSuccess) {
        potato_destroy(ctx);
        return hip_fail(e, "potato_create");
    }
    *out = ctx;
    return POTATO_OK;
}

potato_status potato_destroy(potato_ctx* ctx) {
    if (!ctx) return POTATO_OK;
    drop_graphs(ctx);
    if (ctx->d_table) (void)hipFree(ctx->d_table);
    if (ctx->d_rank) (void)hipFree(ctx->d_rank);
    if (ctx->d_radius) (void)hipFree(ctx->d_radius);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
    return POTATO_OK;
}

potato_status potato_set_options(potato_ctx* ctx, const potato_options* opts) {
    if (!ctx || !opts) return fail(POTATO_EINVAL, "ctx and opts must be non-null");
    potato_status s = check_options(*opts);
    if (s != POTATO_OK) return s;
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->opts = *opts;
    drop_graphs(ctx);
    return POTATO_OK;
}

potato_status potato_step(potato_ctx* ctx, const potato_state* state, const potato_params* params,
                          const potato_cmds* cmds, float dt, int64_t n_agents, int32_t n_steps,
                          float* ckpt, int32_t ckpt_every, void* stream) {
    ApiRange range("potato_step");
    potato_status s = validate_step(ctx, state, params, cmds, dt, n_agents, n_steps, ckpt, ckpt_every);
    if (s != POTATO_OK) return s;
    if (n_steps == 0) return POTATO_OK;
    std::lock_guard<std::mutex> g(ctx->mu);
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    Plan P = make_plan(ctx, state, params, cmds, dt, n_agents, ckpt, ckpt_every);
    if (!ctx->opts.use_graph) {
        hipError_t e = enqueue(P, n_steps, hs);
        return e == hipSuccess ? POTATO_OK : hip_fail(e, "potato_step launch");
    }
    std::vector<int64_t> key = graph_key(P, n_steps, dt);
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        if (ctx->graphs.size() >= 64) drop_graphs(ctx);
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipError_t e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        hipError_t le = enqueue(P, n_steps, ctx->cap_stream);
        e = hipStreamEndCapture(ctx->cap_stream, &graph);
        if (le != hipSuccess) { if (graph) (void)hipGraphDestroy(graph); return hip_fail(le, "potato_step capture"); }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        it = ctx->graphs.emplace(key, exec).first;
    }
    hipError_t e = hipGraphLaunch(it->second, hs);
    return e == hipSuccess ? POTATO_OK : hip_fail(e, "hipGraphLaunch");
}

potato_status potato_autotune(potato_ctx* ctx, const potato_state* state, const potato_params* params,
                              const potato_cmds* cmds, float dt, int64_t n_agents, int32_t probe_steps,
                              int32_t ckpt_every, potato_options* best, void* stream) {
    ApiRange range("potato_autotune");
    if (ckpt_every < 0) return fail(POTATO_EINVAL, "ckpt_every must be >= 0");
    /* validation only asks whether checkpoints are written (any non-null
     * pointer stands for the scratch buffer allocated below) */
    potato_status s = validate_step(ctx, state, params, cmds, dt, n_agents, probe_steps,
                                    ckpt_every > 0 ? state->rows : nullptr, ckpt_every);
    if (s != POTATO_OK) return s;
    if (probe_steps < 1) return fail(POTATO_EINVAL, "probe_steps must be >= 1");
    std::lock_guard<std::mutex> g(ctx->mu);
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    /* scratch copy of the state rows and, if given, of the carries; with
     * ckpt_every, checkpoint slots for probe_steps steps */
    const size_t bytes = sizeof(float) * kRows * (size_t)state->ld;
    const size_t cbytes = state->carry ? sizeof(float) * kCarryRows * (size_t)state->carry_ld : 0;
    const size_t kbytes = ckpt_every > 0 ? sizeof(float) * kCkptRows * (size_t)state->ld *
                                               (size_t)((probe_steps + ckpt_every - 1) / ckpt_every)
                                         : 0;
    float* scratch = nullptr;
    hipError_t e = hipMalloc(&scratch, bytes + cbytes + kbytes);
    if (e != hipSuccess) return fail(POTATO_ENOMEM, "autotune scratch: %s", hipGetErrorString(e));
    e = hipMemcpyAsync(scratch, state->rows, bytes, hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess && cbytes)
        e = hipMemcpyAsync(scratch + kRows * state->ld, state->carry, cbytes, hipMemcpyDeviceToDevice, hs);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    potato_state ss{scratch, state->ld, state->carry ? scratch + kRows * state->ld : nullptr, state->carry_ld};
    float* ckpt_scratch = ckpt_every > 0 ? scratch + (bytes + cbytes) / sizeof(float) : nullptr;
    int n_cu = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device);
    Tuned win{256, 100, 0};
    struct Cand { Tuned t; double ms; };
    std::vector<Cand> cands;
    const int blocks[] = {64, 128, 256, 512, 1024};
    /* steps per launch: the candidates up to probe_steps (at least one) */
    std::vector<int> steps_opts;
    for (int S : {25, 50, 100, 200, 500, 1000})
        if (S <= probe_steps || steps_opts.empty()) steps_opts.push_back(std::min(S, probe_steps));
    const potato_options saved = ctx->opts;
    ctx->opts.form = POTATO_FORM_FUSED;
    /* probe_steps steps with one shape, after one untimed launch of it */
    auto probe = [&](const Tuned& t, double& ms_out) -> hipError_t {
        Plan P = make_plan(ctx, &ss, params, cmds, dt, n_agents, ckpt_scratch, ckpt_every);
        P.block = t.block; P.steps = t.steps; P.grid = t.grid;
        hipError_t pe = enqueue(P, P.steps, hs);
        if (pe == hipSuccess) pe = hipEventRecord(t0, hs);
        if (pe == hipSuccess) pe = enqueue(P, probe_steps, hs);
        if (pe == hipSuccess) pe = hipEventRecord(t1, hs);
        if (pe == hipSuccess) pe = hipEventSynchronize(t1);
        float ms = 0.0f;
        if (pe == hipSuccess) pe = hipEventElapsedTime(&ms, t0, t1);
        ms_out = ms;
        return pe;
    };
    /* the engine clock ramps up over the first launches of a busy GPU (2.0
     * to 2.4 GHz over some tens of milliseconds at 1M agents): three untimed
     * trials of a middle shape first, so that the candidates are timed at
     * the clock they will run at */
    for (int r = 0; r < 3 && e == hipSuccess; ++r) {
        double ms = 0.0;
        e = probe(Tuned{256, steps_opts.back(), 0}, ms);
    }
    for (int b : blocks) {
        if (e != hipSuccess) break;
        Plan P = make_plan(ctx, &ss, params, cmds, dt, n_agents, ckpt_scratch, ckpt_every);
        int per_cu = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, rollout_kernel(P.v), b,
                                                         rollout_lds_bytes(P.v, P.a, b));
        if (e != hipSuccess) break;
        const int64_t full = (n_agents + b - 1) / b;
        std::vector<int> grids = {0};
        for (int mult : {1, 2}) {
            const int64_t gsz = (int64_t)per_cu * n_cu * mult;
            if (gsz > 0 && gsz < full) grids.push_back((int)gsz);
        }
        for (int S : steps_opts) {
            for (int gsz : grids) {
                const Tuned t{b, std::min(S, probe_steps), gsz};
                double ms = 0.0;
                e = probe(t, ms);
                if (e != hipSuccess) break;
                cands.push_back(Cand{t, ms});
            }
            if (e != hipSuccess) break;
        }
    }
    /* Shapes within a few per cent of each other trade places from one
     * probe to the next, so the three fastest are probed three more times,
     * in turn, and the one with the lowest time of those runs wins. */
    if (e == hipSuccess && !cands.empty()) {
        std::sort(cands.begin(), cands.end(), [](const Cand& a, const Cand& b) { return a.ms < b.ms; });
        const size_t top = std::min<size_t>(3, cands.size());
        std::vector<double> best_ms(top, 1e300);
        for (int r = 0; r < 3 && e == hipSuccess; ++r)
            for (size_t c = 0; c < top && e == hipSuccess; ++c) {
                double ms = 0.0;
                e = probe(cands[c].t, ms);
                best_ms[c] = std::min(best_ms[c], ms);
            }
        size_t w = 0;
        for (size_t c = 1; c < top; ++c)
            if (best_ms[c] < best_ms[w]) w = c;
        win = cands[w].t;
    }
    ctx->opts = saved;
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    (void)hipStreamSynchronize(hs);
    (void)hipFree(scratch);
    if (e != hipSuccess) return hip_fail(e, "potato_autotune");
    const bool het = params->type != nullptr;
    ctx->tuned[TuneKey{ctx->opts.mode, het, ctx->opts.mode == 1 && params->gains != nullptr,
                       het && params->perm != nullptr, ckpt_every > 0}] = win;
    drop_graphs(ctx);
    if (best) {
        *best = ctx->opts;
        best->form = POTATO_FORM_FUSED;
        best->block = win.block;
        best->steps_per_launch = win.steps;
        best->grid_blocks = win.grid;
    }
    return POTATO_OK;
}

namespace {

/* Launch shape of the adjoint.  One agent per thread, with enough resident
 * blocks to fill the chip and never more than the agents need; or, when
 * that would leave more than half of the resident wave slots empty (the
 * reverse sweep is latency bound, so a SIMD needs two waves), the
 * pipelined kernel whose recomputing and reversing waves serve the same 64
 * agents (two waves per 64 agents). */
struct AdjShape {
    bool pipe;
    int block;
    int grid;
};

bool adjoint_shape(potato_ctx* ctx, bool het, bool gains, bool perm, int64_t n, AdjShape& out) {
    int per_cu = 0, per_cu_pipe = 0, n_cu = 0;
    const size_t lds = adjoint_lds_bytes(het, ctx->n_types);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, adjoint_kernel(het, gains, perm, false), kAdjBlock,
                                                     lds) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_pipe, adjoint_kernel(het, gains, perm, true),
                                                     kAdjPipeBlock, lds) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess)
        return false;
    n_cu = std::max(n_cu, 1);
    const int64_t resident = (int64_t)std::max(per_cu, 1) * n_cu;
    const int64_t wave_slots = resident * (kAdjBlock / 64);
    const int64_t groups = (n + 63) / 64;                    /* waves of the one-agent-per-thread kernel */
    if (POTATO_ADJOINT_PIPE && 2 * groups <= wave_slots) {
        const int64_t resident_pipe = (int64_t)std::max(per_cu_pipe, 1) * n_cu;
        out = AdjShape{true, kAdjPipeBlock, (int)std::min(resident_pipe, groups)};
    } else {
        out = AdjShape{false, kAdjBlock, (int)std::min(resident, (n + kAdjBlock - 1) / kAdjBlock)};
    }
    return true;
}

int64_t adjoint_tape_bytes(const AdjShape& sh, int32_t ckpt_every) {
    return (int64_t)ckpt_every * kTapeRows * (int64_t)sh.grid * sh.block * (int64_t)sizeof(float);
}

}  // namespace

int64_t potato_backward_workspace_bytes(potato_ctx* ctx, const potato_params* params, int64_t n_agents,
                                        int32_t ckpt_every) {
    if (!ctx || !params || n_agents < 1 || ckpt_every < 1) return -1;
    const bool het = params->type != nullptr;
    AdjShape sh;
    if (!adjoint_shape(ctx, het, params->gains != nullptr, het && params->perm != nullptr, n_agents, sh)) return -1;
    return adjoint_tape_bytes(sh, ckpt_every);
}

potato_status potato_step_backward(potato_ctx* ctx, const potato_params* params, const potato_cmds* cmds,
                                   float dt, int64_t n_agents, int32_t n_steps, const float* ckpt,
                                   int32_t ckpt_every, int64_t ld, const float* grad_final, float* grad_x0,
                                   float* grad_mem, float* grad_gains, void* workspace, int64_t workspace_bytes,
                                   void* stream) {
    ApiRange range("potato_step_backward");
    if (!ctx || !params || !cmds) return fail(POTATO_EINVAL, "ctx, params and cmds must be non-null");
    if (ctx->opts.mode != POTATO_CLOSED_LOOP)
        return fail(POTATO_EUNSUPPORTED, "the adjoint is implemented for closed-loop rollouts");
    if (ctx->kinds)
        return fail(POTATO_EUNSUPPORTED, "the adjoint covers quadrotors only; the type table holds cars or "
                                         "fixed-wing aircraft");
    if (!ckpt || !grad_final || !grad_x0 || !workspace)
        return fail(POTATO_EINVAL, "ckpt, grad_final, grad_x0 and workspace must be non-null");
    if (n_agents < 1 || n_agents > kMaxAgents) return fail(POTATO_EINVAL, "n_agents must be in [1, 2^30]");
    if (ld < n_agents) return fail(POTATO_EINVAL, "ld < n_agents");
    if (n_steps < 0) return fail(POTATO_EINVAL, "n_steps must be >= 0");
    if (ckpt_every < 1) return fail(POTATO_EINVAL, "ckpt_every must be >= 1");
    if (!std::isfinite(dt) || !(dt > 0.0f)) return fail(POTATO_EINVAL, "dt must be finite and > 0");
    if (!cmds->wp || cmds->n_epochs < 1 || cmds->ld < n_agents || cmds->step0 < 0)
        return fail(POTATO_EINVAL, "closed loop needs cmds.wp, n_epochs >= 1, cmds.ld >= n_agents, step0 >= 0");
    if (params->gains && params->gains_ld < n_agents) return fail(POTATO_EINVAL, "params.gains_ld < n_agents");
    if (!params->type && params->perm) return fail(POTATO_EUNSUPPORTED, "params.perm needs params.type");
    const bool het = params->type != nullptr;
    const bool gains = params->gains != nullptr;
    const bool perm = het && params->perm != nullptr;
    std::lock_guard<std::mutex> g(ctx->mu);
    AdjShape sh;
    if (!adjoint_shape(ctx, het, gains, perm, n_agents, sh)) return fail(POTATO_EHIP, "occupancy query failed");
    const int64_t need = adjoint_tape_bytes(sh, ckpt_every);
    if (workspace_bytes < need)
        return fail(POTATO_EINVAL, "workspace too small: need %lld bytes", (long long)need);
    AdjArgs a{};
    a.ckpt = ckpt; a.ld = ld; a.n = n_agents;
    a.type = params->type; a.perm = perm ? params->perm : nullptr;
    a.gains = params->gains; a.gains_ld = params->gains_ld;
    a.wp = cmds->wp; a.cmd_ld = cmds->ld; a.n_epochs = cmds->n_epochs; a.resample = cmds->resample_every;
    a.step0 = cmds->step0; a.n_steps = n_steps; a.K = ckpt_every;
    a.grad_final = grad_final; a.grad_x0 = grad_x0; a.grad_mem = grad_mem; a.grad_gains = grad_gains;
    a.tape = reinterpret_cast<float*>(workspace); a.tape_ld = (int64_t)sh.grid * sh.block;
    a.n_types = het ? ctx->n_types : 1; a.table = ctx->d_table;
    a.alive = params->alive;
    a.lim = make_limits(ctx->limits, dt);
    hipError_t e = launch_adjoint(het, gains, perm, sh.pipe, a, sh.grid, reinterpret_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipGetLastError();
    return e == hipSuccess ? POTATO_OK : hip_fail(e, "potato_step_backward launch");
}

int64_t potato_order_workspace_bytes(int64_t n_agents, int32_t n_types) {
    if (n_agents < 1 || n_types < 1 || n_types > POTATO_MAX_TYPES) return -1;
    return order_workspace_words(n_agents, n_types) * (int64_t)sizeof(int32_t);
}

potato_status potato_order_by_type(potato_ctx* ctx, const uint8_t* type, int64_t n_agents, int32_t* perm,
                                   void* workspace, int64_t workspace_bytes, void* stream) {
    ApiRange range("potato_order_by_type");
    if (!ctx || !type || !perm || !workspace) return fail(POTATO_EINVAL, "ctx, type, perm and workspace must be non-null");
    if (n_agents < 1 || n_agents > kMaxAgents) return fail(POTATO_EINVAL, "n_agents must be in [1, 2^30]");
    const int64_t need = potato_order_workspace_bytes(n_agents, ctx->n_types);
    if (workspace_bytes < need) return fail(POTATO_EINVAL, "workspace too small: need %lld bytes", (long long)need);
    hipError_t e = launch_order_by_type(type, n_agents, ctx->n_types, ctx->d_rank, perm,
                                        reinterpret_cast<int32_t*>(workspace),
                                        reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? POTATO_OK : hip_fail(e, "potato_order_by_type");
}

int64_t potato_collision_workspace_bytes(int64_t n_agents) {
    if (n_agents < 1 || n_agents > 0x3fffffffLL) return -1;
    return collision_workspace_bytes(n_agents);
}

namespace {

potato_status detect_collisions(const char* name, potato_ctx* ctx, const potato_state* state,
                                const potato_params* params, int64_t n_agents, uint8_t* alive, int64_t* died,
                                void* workspace, void* stream) {
    hipError_t e = launch_detect_collisions(state->rows, state->ld, n_agents, params ? params->type : nullptr,
                                            ctx->n_types, ctx->d_radius, ctx->r_max, alive,
                                            reinterpret_cast<unsigned long long*>(died), workspace,
                                            reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? POTATO_OK : hip_fail(e, name);
}

potato_status check_collision_args(const potato_ctx* ctx, const potato_state* state, int64_t n_agents,
                                   const uint8_t* alive) {
    if (!ctx || !state || !state->rows || !alive)
        return fail(POTATO_EINVAL, "ctx, state, state.rows and alive must be non-null");
    if (n_agents < 1 || n_agents > 0x3fffffffLL) return fail(POTATO_EINVAL, "n_agents must be in [1, 2^30)");
    if (state->ld < n_agents) return fail(POTATO_EINVAL, "state.ld < n_agents");
    if (!(ctx->r_max > 0.0f)) return fail(POTATO_EINVAL, "every type has radius 0: nothing can collide");
    return POTATO_OK;
}

}  // namespace

potato_status potato_detect_collisions(potato_ctx* ctx, const potato_state* state, const potato_params* params,
                                       int64_t n_agents, uint8_t* alive, int64_t* died, void* workspace,
                                       int64_t workspace_bytes, void* stream) {
    ApiRange range("potato_detect_collisions");
    potato_status s = check_collision_args(ctx, state, n_agents, alive);
    if (s != POTATO_OK) return s;
    if (!workspace) return fail(POTATO_EINVAL, "workspace must be non-null");
    const int64_t need = collision_workspace_bytes(n_agents);
    if (workspace_bytes < need) return fail(POTATO_EINVAL, "workspace too small: need %lld bytes", (long long)need);
    return detect_collisions("potato_detect_collisions launch", ctx, state, params, n_agents, alive, died,
                             workspace, stream);
}

potato_status potato_detect_collisions_noalloc(potato_ctx* ctx, const potato_state* state,
                                               const potato_params* params, int64_t n_agents, uint8_t* alive,
                                               int64_t* died, void* stream) {
    ApiRange range("potato_detect_collisions_noalloc");
    potato_status s = check_collision_args(ctx, state, n_agents, alive);
    if (s != POTATO_OK) return s;
    if (n_agents > kNoAllocMaxAgents)
        return fail(POTATO_EINVAL, "n_agents (%lld) exceeds the static workspace's limit of %lld agents",
                    (long long)n_agents, (long long)kNoAllocMaxAgents);
    if (!ctx->scratch || ctx->scratch_bytes < collision_workspace_bytes(n_agents))
        return fail(POTATO_EHIP, "static collision workspace unavailable on this device");
    return detect_collisions("potato_detect_collisions_noalloc launch", ctx, state, params, n_agents, alive, died,
                             ctx->scratch, stream);
}

potato_status potato_count_nonfinite(potato_ctx* ctx, const potato_state* state, int64_t n_agents, int64_t* count,
                                     void* stream) {
    ApiRange range("potato_count_nonfinite");
    if (!ctx || !state || !state->rows || !count)
        return fail(POTATO_EINVAL, "ctx, state, state.rows and count must be non-null");
    if (n_agents < 1 || n_agents > kMaxAgents) return fail(POTATO_EINVAL, "n_agents must be in [1, 2^30]");
    if (state->ld < n_agents) return fail(POTATO_EINVAL, "state.ld < n_agents");
    const int n_rows = ctx->opts.mode == POTATO_CLOSED_LOOP ? 30 : 17;
    hipError_t e = launch_count_nonfinite(state->rows, state->ld, n_agents, n_rows,
                                          reinterpret_cast<unsigned long long*>(count),
                                          reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? POTATO_OK : hip_fail(e, "potato_count_nonfinite launch");
}

const char* potato_last_error(const potato_ctx*) { return g_err.c_str(); }

const char* potato_version(void) { return "potato-mi355x 0.1 (gfx950)"; }

}  // extern "C"
