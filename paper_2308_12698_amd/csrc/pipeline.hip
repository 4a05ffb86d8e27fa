/*
 * pipeline.hip -- command ingress and position snapshots overlapped with a
 * running rollout (the decision and viewer directions of the system of
 * Sec. II-A, Fig. 2, which the paper keeps outside the simulation loop).
 *
 * Streams and ordering.  Runs go to the caller's compute stream.  Command
 * uploads go to the pipe's ingress stream, snapshot downloads to its egress
 * stream, so neither waits behind the other.  Every cross-stream wait names
 * an event recorded earlier in host order, so the three streams cannot wait
 * on each other in a cycle:
 *   push k  (slot s = k mod 2):  ingress waits "slot s read" (the last run
 *           that used slot s), uploads, records "slot s ready";
 *   run     (slot of the last push): compute waits "slot ready", runs,
 *           records "slot read";
 *   snapshot j, direct (host_snap is pinned host memory mapped into the
 *           device's address space): the last launch before the snapshot
 *           writes every agent's position straight into host_snap as its
 *           waves finish, so the PCIe writes overlap the other waves' work;
 *           compute records "taken", egress waits it and records
 *           landed[j mod kRing];
 *   snapshot j, copied (any other host memory; slot t = j mod 2): compute
 *           waits "snapshot slot t free" (the download of snapshot j-2),
 *           copies rows 0-2 into slot t, records "slot t taken"; egress
 *           waits it, downloads, records "snapshot slot t free" and
 *           landed[j mod kRing].
 * Both kinds record landed[] on the egress stream, so snapshots land in
 * order whichever way each one went.  Everything the pipe uses is
 * allocated at creation.
 */
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>

#include "../../include/potato.h"
#include "internal.h"

using namespace potato;

namespace {
constexpr int kRing = 64;   /* snapshot completion events kept for waits */
}

struct potato_pipe {
    potato_ctx* ctx = nullptr;
    int64_t n = 0;
    int rows = 0;                      /* 3 waypoint rows or 4 rotor-command rows */
    int mode = 0;
    hipStream_t ingress = nullptr, egress = nullptr;
    hipStream_t run_stream = nullptr;
    bool have_run_stream = false;
    float* d_cmd[2] = {nullptr, nullptr};
    float* h_cmd[2] = {nullptr, nullptr};
    float* d_snap[2] = {nullptr, nullptr};
    hipEvent_t cmd_ready[2] = {}, cmd_read[2] = {}, snap_taken[2] = {}, snap_free[2] = {};
    bool cmd_uploaded[2] = {false, false}, cmd_was_read[2] = {false, false}, snap_used[2] = {false, false};
    hipEvent_t landed[kRing] = {};
    int64_t pushed = 0;
    int64_t snaps = 0;                 /* snapshots enqueued since creation */
    int64_t direct = 0;                /* of which written straight to mapped host memory */
    int64_t step = 0;                  /* global index of the next step */
};

namespace {

void release(potato_pipe* p) {
    if (p->have_run_stream) (void)hipStreamSynchronize(p->run_stream);
    if (p->ingress) (void)hipStreamSynchronize(p->ingress);
    if (p->egress) (void)hipStreamSynchronize(p->egress);
    for (int s = 0; s < 2; ++s) {
        if (p->d_cmd[s]) (void)hipFree(p->d_cmd[s]);
        if (p->h_cmd[s]) (void)hipHostFree(p->h_cmd[s]);
        if (p->d_snap[s]) (void)hipFree(p->d_snap[s]);
        for (hipEvent_t ev : {p->cmd_ready[s], p->cmd_read[s], p->snap_taken[s], p->snap_free[s]})
            if (ev) (void)hipEventDestroy(ev);
    }
    for (hipEvent_t ev : p->landed)
        if (ev) (void)hipEventDestroy(ev);
    if (p->ingress) (void)hipStreamDestroy(p->ingress);
    if (p->egress) (void)hipStreamDestroy(p->egress);
    delete p;
}

hipError_t make_event(hipEvent_t* ev) { return hipEventCreateWithFlags(ev, hipEventDisableTiming); }

/* Device view of `host` if it is pinned host memory that the device
 * addresses at the same virtual address (ROCm maps hipHostMalloc memory
 * so); null for pageable memory or when the allocation's extent is
 * unknown.  *short_range is set when the allocation ends before
 * host + bytes. */
float* mapped_view(float* host, size_t bytes, bool* short_range) {
    *short_range = false;
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, host) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (at.type != hipMemoryTypeHost || !at.devicePointer || at.devicePointer != at.hostPointer) return nullptr;
    void* base = nullptr;
    size_t size = 0;
    if (hipPointerGetAttribute(&base, HIP_POINTER_ATTRIBUTE_RANGE_START_ADDR, host) != hipSuccess ||
        hipPointerGetAttribute(&size, HIP_POINTER_ATTRIBUTE_RANGE_SIZE, host) != hipSuccess || !base || !size) {
        (void)hipGetLastError();
        return nullptr;
    }
    const uintptr_t b = reinterpret_cast<uintptr_t>(base), h = reinterpret_cast<uintptr_t>(host);
    if (h < b || h - b > size || size - (h - b) < bytes) {
        *short_range = true;
        return nullptr;
    }
    return host;
}

}  // namespace

extern "C" {

potato_status potato_pipe_create(potato_ctx* ctx, int64_t n_agents, potato_pipe** out) {
    if (!out) return set_error(POTATO_EINVAL, "out is null");
    *out = nullptr;
    if (!ctx) return set_error(POTATO_EINVAL, "ctx is null");
    if (n_agents < 1 || n_agents > (int64_t(1) << 30)) return set_error(POTATO_EINVAL, "n_agents must be in [1, 2^30]");
    potato_pipe* p = new (std::nothrow) potato_pipe();
    if (!p) return set_error(POTATO_ENOMEM, "host allocation failed");
    p->ctx = ctx;
    p->n = n_agents;
    p->mode = ctx_mode(ctx);
    p->rows = p->mode == POTATO_CLOSED_LOOP ? 3 : 4;
    const size_t cmd_bytes = sizeof(float) * p->rows * (size_t)n_agents;
    const size_t snap_bytes = sizeof(float) * 3 * (size_t)n_agents;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess && dev != ctx_device(ctx)) {
        release(p);
        return set_error(POTATO_EINVAL, "the current device is not the context's device");
    }
    /* default-priority streams that do not synchronise with the null stream */
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->ingress, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->egress, hipStreamNonBlocking);
    for (int s = 0; s < 2 && e == hipSuccess; ++s) {
        e = hipMalloc(&p->d_cmd[s], cmd_bytes);
        if (e == hipSuccess) e = hipHostMalloc(&p->h_cmd[s], cmd_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc(&p->d_snap[s], snap_bytes);
        if (e == hipSuccess) e = make_event(&p->cmd_ready[s]);
        if (e == hipSuccess) e = make_event(&p->cmd_read[s]);
        if (e == hipSuccess) e = make_event(&p->snap_taken[s]);
        if (e == hipSuccess) e = make_event(&p->snap_free[s]);
    }
    for (int r = 0; r < kRing && e == hipSuccess; ++r) e = make_event(&p->landed[r]);
    if (e != hipSuccess) {
        release(p);
        return e == hipErrorOutOfMemory ? set_error(POTATO_ENOMEM, "potato_pipe_create: out of memory")
                                        : set_hip_error(e, "potato_pipe_create");
    }
    *out = p;
    return POTATO_OK;
}

potato_status potato_pipe_push(potato_pipe* p, const float* host_cmd) {
    ApiRange range("potato_pipe_push");
    if (!p || !host_cmd) return set_error(POTATO_EINVAL, "pipe and host_cmd must be non-null");
    const int s = (int)(p->pushed & 1);
    const size_t bytes = sizeof(float) * p->rows * (size_t)p->n;
    hipError_t e = hipSuccess;
    /* the staging slot is reused only after its previous upload finished */
    if (p->cmd_uploaded[s]) e = hipEventSynchronize(p->cmd_ready[s]);
    if (e != hipSuccess) return set_hip_error(e, "potato_pipe_push (wait for staging slot)");
    std::memcpy(p->h_cmd[s], host_cmd, bytes);
    if (p->cmd_was_read[s]) e = hipStreamWaitEvent(p->ingress, p->cmd_read[s], 0);
    if (e == hipSuccess) e = hipMemcpyAsync(p->d_cmd[s], p->h_cmd[s], bytes, hipMemcpyHostToDevice, p->ingress);
    if (e == hipSuccess) e = hipEventRecord(p->cmd_ready[s], p->ingress);
    if (e != hipSuccess) return set_hip_error(e, "potato_pipe_push");
    p->cmd_uploaded[s] = true;
    p->pushed += 1;
    return POTATO_OK;
}

potato_status potato_pipe_run(potato_pipe* p, const potato_state* state, const potato_params* params, float dt,
                              int32_t n_steps, int32_t snap_every, float* host_snap, void* stream) {
    ApiRange range("potato_pipe_run");
    if (!p || !state || !params) return set_error(POTATO_EINVAL, "pipe, state and params must be non-null");
    if (p->pushed < 1) return set_error(POTATO_EINVAL, "potato_pipe_run before the first potato_pipe_push");
    if (n_steps < 0 || snap_every < 0) return set_error(POTATO_EINVAL, "n_steps and snap_every must be >= 0");
    if (snap_every > 0 && n_steps >= snap_every && !host_snap)
        return set_error(POTATO_EINVAL, "host_snap is null but a snapshot is due");
    if (ctx_mode(p->ctx) != p->mode)
        return set_error(POTATO_EINVAL, "the context's mode changed since the pipe was created");
    if (!state->rows || state->ld < p->n) return set_error(POTATO_EINVAL, "state.rows null or state.ld < n_agents");
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    if (p->have_run_stream && hs != p->run_stream)
        return set_error(POTATO_EINVAL, "every run of a pipe must use the same stream");
    if (n_steps == 0) return POTATO_OK;
    p->run_stream = hs;
    p->have_run_stream = true;

    const int cur = (int)((p->pushed - 1) & 1);
    potato_cmds cmds{};
    if (p->mode == POTATO_CLOSED_LOOP) {
        cmds.wp = p->d_cmd[cur];
        cmds.n_epochs = 1;
    } else {
        cmds.motor_cmd = p->d_cmd[cur];
    }
    cmds.resample_every = 0;
    cmds.ld = p->n;
    hipError_t e = hipStreamWaitEvent(hs, p->cmd_ready[cur], 0);
    if (e != hipSuccess) return set_hip_error(e, "potato_pipe_run (wait for commands)");

    const int32_t seg = snap_every > 0 ? snap_every : n_steps;
    const size_t row_bytes = sizeof(float) * (size_t)p->n;
    const size_t snap_bytes = 3 * row_bytes;
    const int64_t due = snap_every > 0 ? n_steps / snap_every : 0;
    float* view = nullptr;
    if (due > 0) {
        bool short_range = false;
        view = mapped_view(host_snap, (size_t)due * snap_bytes, &short_range);
        if (short_range)
            return set_error(POTATO_EINVAL, "host_snap's allocation holds fewer than the %lld snapshots due",
                             (long long)due);
    }
    int64_t k = 0;   /* snapshot index within this run */
    for (int32_t k0 = 0; k0 < n_steps; k0 += seg) {
        const int32_t len = std::min(seg, n_steps - k0);
        const bool snapshot = snap_every > 0 && len == snap_every;
        float* direct = snapshot && view ? view + k * 3 * p->n : nullptr;
        cmds.step0 = p->step;
        potato_status st = step_eager(p->ctx, state, params, &cmds, dt, p->n, len, hs, direct);
        if (st != POTATO_OK) return st;
        p->step += len;
        if (!snapshot) continue;
        const int t = (int)(p->snaps & 1);
        if (direct) {
            e = hipEventRecord(p->snap_taken[t], hs);
            if (e == hipSuccess) e = hipStreamWaitEvent(p->egress, p->snap_taken[t], 0);
            if (e == hipSuccess) e = hipEventRecord(p->landed[p->snaps % kRing], p->egress);
            if (e != hipSuccess) return set_hip_error(e, "potato_pipe_run (snapshot)");
            p->snaps += 1;
            p->direct += 1;
            k += 1;
            continue;
        }
        if (p->snap_used[t]) e = hipStreamWaitEvent(hs, p->snap_free[t], 0);
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(p->d_snap[t], row_bytes, state->rows, sizeof(float) * (size_t)state->ld, row_bytes,
                                 3, hipMemcpyDeviceToDevice, hs);
        if (e == hipSuccess) e = hipEventRecord(p->snap_taken[t], hs);
        if (e == hipSuccess) e = hipStreamWaitEvent(p->egress, p->snap_taken[t], 0);
        if (e == hipSuccess)
            e = hipMemcpyAsync(host_snap + k * 3 * p->n, p->d_snap[t], snap_bytes, hipMemcpyDeviceToHost, p->egress);
        if (e == hipSuccess) e = hipEventRecord(p->snap_free[t], p->egress);
        if (e == hipSuccess) e = hipEventRecord(p->landed[p->snaps % kRing], p->egress);
        if (e != hipSuccess) return set_hip_error(e, "potato_pipe_run (snapshot)");
        p->snap_used[t] = true;
        p->snaps += 1;
        k += 1;
    }
    e = hipEventRecord(p->cmd_read[cur], hs);
    if (e != hipSuccess) return set_hip_error(e, "potato_pipe_run");
    p->cmd_was_read[cur] = true;
    return POTATO_OK;
}

potato_status potato_pipe_wait_snapshots(potato_pipe* p, int64_t count) {
    ApiRange range("potato_pipe_wait_snapshots");
    if (!p) return set_error(POTATO_EINVAL, "pipe is null");
    if (count < 0 || count > p->snaps)
        return set_error(POTATO_EINVAL, "count must be in [0, %lld] (snapshots enqueued)", (long long)p->snaps);
    if (count == 0) return POTATO_OK;
    /* downloads complete in order on the egress stream; if the event of
     * snapshot count-1 was reused, the oldest live one is a later snapshot */
    const int64_t j = std::max(count - 1, p->snaps - kRing);
    hipError_t e = hipEventSynchronize(p->landed[j % kRing]);
    return e == hipSuccess ? POTATO_OK : set_hip_error(e, "potato_pipe_wait_snapshots");
}

potato_status potato_pipe_sync(potato_pipe* p) {
    ApiRange range("potato_pipe_sync");
    if (!p) return set_error(POTATO_EINVAL, "pipe is null");
    hipError_t e = hipStreamSynchronize(p->ingress);
    if (e == hipSuccess) e = hipStreamSynchronize(p->egress);
    return e == hipSuccess ? POTATO_OK : set_hip_error(e, "potato_pipe_sync");
}

potato_status potato_pipe_stats(const potato_pipe* p, int64_t* snapshots, int64_t* direct) {
    if (!p || !snapshots || !direct) return set_error(POTATO_EINVAL, "pipe, snapshots and direct must be non-null");
    *snapshots = p->snaps;
    *direct = p->direct;
    return POTATO_OK;
}

potato_status potato_pipe_destroy(potato_pipe* p) {
    if (!p) return POTATO_OK;
    release(p);
    return POTATO_OK;
}

}  // extern "C"
