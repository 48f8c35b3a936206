// fse_graph.cpp -- prepared plans replayed as HIP graphs.
//
// When the loss masks stay the same over many images (a sensor's defect map
// over a video, a fixed logo), the block planning, dependency order and
// device tables depend only on the masks.  A plan does that work once, keeps
// private copies of the masks and its own working state, and captures the
// launch sequence -- an upload of the per-image pointer table from pinned
// host memory, the state-initialisation kernel and the persistent block
// kernel -- into one HIP graph.  Each execution updates the pinned pointer
// table and replays the graph.  The graph holds no memset node: counters and
// flags are cleared by the initialisation kernel.
#include <hip/hip_runtime.h>

#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/fse.h"
#include "fse_internal.h"
#include "fse_plan.h"
#include "fse_runtime.h"

struct fse_plan {
    std::mutex mu;
    int n = 0;
    std::vector<int> width, height;
    std::vector<uint8_t*> mask_copy;  // private device copies of the masks
    fse_params_t params{};
    fse::Workspace ws;
    fse::Prepared P;
    hipStream_t stream = nullptr;  // stream the graph was captured on
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;  // completion of the last execution
    bool launched = false;
};

namespace {

void destroy_plan(fse_plan* P) {
    if (!P) return;
    if (P->launched && P->done) (void)hipEventSynchronize(P->done);
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->done) (void)hipEventDestroy(P->done);
    if (P->stream) (void)hipStreamDestroy(P->stream);
    for (uint8_t* m : P->mask_copy)
        if (m) (void)hipFree(m);
    P->ws.free_all();
    delete P;
}

}  // namespace

using fse::abi_guard;

extern "C" {

fse_status_t fse_plan_create(int32_t n, const fse_mask_t* masks, const fse_params_t* p, fse_plan_t** plan) {
    return abi_guard([&]() -> fse_status_t {
        using namespace fse;
        if (n < 1 || !masks || !p || !plan) return FSE_ERR_INVALID_ARG;
        if (p->schedule != FSE_SCHED_PERSISTENT || p->trace_sel) return FSE_ERR_INVALID_ARG;
        std::vector<ClassCfg> cls;
        fse_status_t s = check_params(p, cls);
        if (s != FSE_OK) return s;
        for (int i = 0; i < n; ++i)
            if (!masks[i].data || masks[i].width < 1 || masks[i].height < 1 || masks[i].pitch < masks[i].width)
                return FSE_ERR_INVALID_ARG;
        // destroyed on every early return (and on an exception)
        std::unique_ptr<fse_plan, void (*)(fse_plan*)> holder(new fse_plan(), destroy_plan);
        fse_plan* P = holder.get();
        P->n = n;
        P->params = *p;
        hipError_t e = hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&P->done, hipEventDisableTiming);
        std::vector<fse_mask_t> own(n);
        std::vector<fse_image_t> img(n), out(n);
        for (int i = 0; e == hipSuccess && i < n; ++i) {
            const int W = masks[i].width, H = masks[i].height;
            P->width.push_back(W);
            P->height.push_back(H);
            uint8_t* m = nullptr;
            e = hipMalloc(&m, (size_t)W * H);
            P->mask_copy.push_back(m);
            if (e == hipSuccess)
                e = hipMemcpy2DAsync(m, W, masks[i].data, masks[i].pitch, W, H, hipMemcpyDeviceToDevice, P->stream);
            own[i] = {m, W, H, W};
            // placeholder image pointers (distinct and non-null); every execution
            // writes the real ones into the pinned pointer table before replaying
            img[i] = {reinterpret_cast<float*>(16 * (2 * i + 1)), W, H, W};
            out[i] = {reinterpret_cast<float*>(16 * (2 * i + 2)), W, H, W};
        }
        if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
        if (e != hipSuccess) return from_hip(e);
        s = prepare_batch(P->ws, n, img.data(), own.data(), p, out.data(), cls, P->stream, P->P);
        if (s == FSE_OK && hipStreamSynchronize(P->stream) != hipSuccess) s = FSE_ERR_DEVICE;
        if (s != FSE_OK) return s;
        // capture: pointer table upload, state initialisation, persistent kernel
        e = hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess)
            e = hipMemcpyAsync(P->ws.jobs.p, P->ws.stage + P->P.o_jobs, P->P.b_jobs, hipMemcpyHostToDevice, P->stream);
        fse_status_t ls = FSE_OK;
        if (e == hipSuccess) ls = launch_prepared(P->ws, P->P, P->stream, false);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(P->stream, &g);
        P->graph = g;
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess && ls == FSE_OK) e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
        if (e != hipSuccess || ls != FSE_OK) return e != hipSuccess ? from_hip(e) : ls;
        *plan = holder.release();
        return FSE_OK;
    });
}

fse_status_t fse_plan_execute(fse_plan_t* P, const fse_image_t* images, fse_image_t* outs, void* stream) {
    return abi_guard([&]() -> fse_status_t {
        using namespace fse;
        if (!P || !images || !outs) return FSE_ERR_INVALID_ARG;
        for (int i = 0; i < P->n; ++i) {
            const fse_image_t& a = images[i];
            const fse_image_t& o = outs[i];
            if (!a.data || !o.data || a.data == o.data || a.width != P->width[i] || a.height != P->height[i] ||
                o.width != P->width[i] || o.height != P->height[i] || a.pitch < a.width || o.pitch < o.width)
                return FSE_ERR_INVALID_ARG;
        }
        std::lock_guard<std::mutex> lk(P->mu);
        // the previous execution must have consumed the pinned pointer table
        if (P->launched) {
            const hipError_t e = hipEventSynchronize(P->done);
            if (e != hipSuccess) return from_hip(e);
        }
        JobDev* jobs = reinterpret_cast<JobDev*>(P->ws.stage + P->P.o_jobs);
        for (int j = 0; j < P->P.n_jobs; ++j) {
            const int i = P->P.job_image[j];
            jobs[j].img = images[i].data;
            jobs[j].img_pitch = images[i].pitch;
            jobs[j].out = outs[i].data;
            jobs[j].out_pitch = outs[i].pitch;
        }
        hipStream_t st = (hipStream_t)stream;
        hipError_t e = hipGraphLaunch(P->exec, st);
        if (e == hipSuccess) e = hipEventRecord(P->done, st);
        if (e != hipSuccess) return from_hip(e);
        P->launched = true;
        return FSE_OK;
    });
}

fse_status_t fse_plan_stats(fse_plan_t* P, fse_run_stats_t* st) {
    return abi_guard([&]() -> fse_status_t {
        using namespace fse;
        if (!P || !st) return FSE_ERR_INVALID_ARG;
        std::lock_guard<std::mutex> lk(P->mu);
        fse_run_stats_t r = P->P.stats;
        r.kernel_ms = 0.0;  // graph launches are not timed
        r.device_error = 0;
        r.n_degenerate = 0;
        if (P->launched) {
            hipError_t e = hipEventSynchronize(P->done);
            // the plan's own stream is idle: the copy runs at once
            int32_t misc[4] = {0, 0, 0, 0};
            if (e == hipSuccess)
                e = hipMemcpyAsync(misc, P->ws.misc.p, sizeof(misc), hipMemcpyDeviceToHost, P->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
            if (e != hipSuccess) return from_hip(e);
            r.device_error = misc[0];
            int64_t deg = 0;
            std::memcpy(&deg, misc + 2, sizeof(deg));
            r.n_degenerate = deg;
        }
        *st = r;
        return FSE_OK;
    });
}

fse_status_t fse_plan_destroy(fse_plan_t* P) {
    return abi_guard([&]() -> fse_status_t {
        if (!P) return FSE_ERR_INVALID_ARG;
        destroy_plan(P);
        return FSE_OK;
    });
}

}  // extern "C"
