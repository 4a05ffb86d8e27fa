/*
 * internal.h -- host-side helpers shared by the translation units of the C
 * ABI (abi.hip, pipeline.hip).  Not installed; not part of the ABI.
 */
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stdint.h>

#include "../../include/potato.h"

namespace potato {

/* A named roctx range over one call of an entry point that enqueues GPU
 * work, so that a marker trace (rocprofv3 --marker-trace) shows which
 * library call each kernel came from.  Without a profiler attached a range
 * costs a call into the roctx library and nothing else. */
struct ApiRange {
    explicit ApiRange(const char* name) { roctxRangePushA(name); }
    ~ApiRange() { roctxRangePop(); }
    ApiRange(const ApiRange&) = delete;
    ApiRange& operator=(const ApiRange&) = delete;
};

/* Record `fmt` as the calling thread's last error and return `st`. */
potato_status set_error(potato_status st, const char* fmt, ...);
potato_status set_hip_error(hipError_t e, const char* where);

/* Mode (open / closed loop) the context was created or last set with. */
int ctx_mode(const potato_ctx* ctx);
int ctx_device(const potato_ctx* ctx);

/* potato_step without hipGraph capture: validates, plans with the tuned
 * launch shape and enqueues the launches on `stream`.  With `snap` (the
 * device view of mapped pinned host memory holding [3][n_agents] floats)
 * the last launch also writes every agent's position there. */
potato_status step_eager(potato_ctx* ctx, const potato_state* state, const potato_params* params,
                         const potato_cmds* cmds, float dt, int64_t n_agents, int32_t n_steps,
                         hipStream_t stream, float* snap = nullptr);

}  // namespace potato
