// fse_runtime.h -- host runtime pieces of libfse: device buffers and the
// per-stream workspace (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <deque>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/fse.h"
#include "fse_internal.h"
#include "fse_plan.h"

namespace fse {

// The body of every C entry point runs inside this guard, so no C++
// exception crosses the ABI: an allocation failure becomes OUT_OF_MEMORY,
// any other exception (a size no container can hold) INVALID_ARG.
template <class F>
fse_status_t abi_guard(F&& body) noexcept {
    try {
        return body();
    } catch (const std::bad_alloc&) {
        return FSE_ERR_OUT_OF_MEMORY;
    } catch (...) {
        return FSE_ERR_INVALID_ARG;
    }
}

// A grow-only device allocation.  Growing retires the old allocation to
// `retired` (freed later, where waiting for the device is acceptable):
// hipFree waits for every stream of the device, which would stall this
// call behind launches of other streams.
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t n, std::vector<void*>& retired);
    void release();
};

// Fixed storage for a workspace that must not allocate: device buffers are
// carved in call order from one device range (reset at every call), and the
// host staging buffers are fixed arrays.  A call that needs more than a range
// holds fails with FSE_ERR_BUDGET before anything is enqueued.
struct Arena {
    unsigned char* dev = nullptr;  // device address of the range
    size_t dev_cap = 0, used = 0;
    uint8_t* host_mask = nullptr;  // mask read-back
    size_t host_mask_cap = 0;
    uint8_t* host_stage = nullptr;  // planning tables before upload
    size_t host_stage_cap = 0;
    hipError_t take(DevBuf& b, size_t n);
};

// Everything one extrapolation call needs on the device.  Calls that use the
// same stream share one workspace and are serialised by its mutex.
struct Workspace {
    std::mutex mu;
    uint64_t gen = 0;  // registry generation: tells a released workspace from a new one on the same stream
    DevBuf recon, owner, desc, lbox, done, tickets, jobs, misc, tabs;
    std::vector<double> tab_key;  // parameters the uploaded tables were built for
    uint8_t* host_mask = nullptr;  // pinned staging for mask read-back
    size_t host_mask_cap = 0;
    uint8_t* stage = nullptr;  // pinned staging for the planning tables
    size_t stage_cap = 0;
    // allocations replaced by larger ones, freed by free_all (device, pinned)
    std::vector<void*> retired_dev, retired_host;
    hipStream_t last_stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;  // bracket the block kernel(s) of the last call
    bool timed = false;
    // host planning state per job, reused between calls
    std::deque<RegionPlan> plans;
    std::vector<PlanScratch> plan_scratch;
    Arena* arena = nullptr;  // set: every buffer comes from the arena (nothing is allocated or freed)
    // a device buffer of at least n bytes: grown (allocating), or carved from the arena
    hipError_t grow(DevBuf& b, size_t n) { return arena ? arena->take(b, n) : b.ensure(n, retired_dev); }
    void free_all();
};

struct ClassCfg;
fse_status_t from_hip(hipError_t e);
fse_status_t check_params(const fse_params_t* p, std::vector<ClassCfg>& cls);
// one extrapolation call (fse_extrapolate / fse_extrapolate_batch)
fse_status_t run_batch(int n, const fse_image_t* images, const fse_mask_t* masks, const fse_params_t* p,
                       fse_image_t* outs, hipStream_t st);
// A planned batch: device tables uploaded into a workspace, ready to launch.
struct Prepared {
    LaunchArgs a{};
    int n_jobs = 0, max_w = 1, max_h = 1, nw = 4, grid = 1, precision = 0, schedule = 0, max_key = 0;
    bool wide = false;
    int64_t ntk = 0;
    std::vector<int32_t> kstart;
    size_t o_jobs = 0, b_jobs = 0;  // the JobDev table inside the workspace's pinned staging
    std::vector<int> job_image;     // image of every job
    fse_run_stats_t stats{};
};
fse_status_t prepare_batch(Workspace& ws, int n, const fse_image_t* images, const fse_mask_t* masks,
                           const fse_params_t* p, const fse_image_t* outs, const std::vector<ClassCfg>& cls,
                           hipStream_t st, Prepared& P);
fse_status_t launch_prepared(Workspace& ws, Prepared& P, hipStream_t st, bool timed);
// record a call of fse_extrapolate_noalloc as this thread's last call
void set_last_call_noalloc(const fse_run_stats_t& st, int dev, hipStream_t s, hipEvent_t done, const int32_t* misc);
// statistics of this thread's last call as planned on the host (no device wait)
void fse_last_stats_nowait(fse_run_stats_t* st);
// The stream's workspace on the current device, returned with its mutex
// held by `lk` (taken while the registry is locked, so a concurrent release
// cannot free it in between).
Workspace* workspace_for(hipStream_t st, std::unique_lock<std::mutex>& lk);
// The error word of the last launch on stream st (its workspace on the
// current device): non-zero when a dependency wait hit its time limit.  The
// launch must have completed.
fse_status_t read_launch_error(hipStream_t st, int32_t* error);
// free the workspace of one stream (before the stream is destroyed)
void release_workspace(int dev, hipStream_t st);
void release_all_workspaces();
int persistent_grid(int nw, int prec, bool wide);  // resident workgroups of the block kernel on the current device

}  // namespace fse
