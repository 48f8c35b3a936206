// fse_serve.cpp -- continuous-batching request server of libfse.
//
// A server owns `max_slots` HIP streams.  Submitted requests wait in a FIFO
// queue.  A scheduler thread repeatedly takes the requests that fit the HBM
// budget (estimated per request from its size), groups those with identical
// parameters, and hands each group to a free stream slot, whose own thread
// plans it on the host and launches it as one batched persistent
// extrapolation (so the planning of several groups runs at once).  Launches on different slots run concurrently on the
// device, so requests that arrive while earlier ones are on the GPU join the
// next launch and overlap with them.  A launch's completion (an event on its
// stream) releases its budget and marks its requests done -- or failed, when
// the launch's error word reports a dependency wait that hit its time limit
// or the event reports a device error.  Results do not
// depend on what else is in a launch: every request keeps its own working
// state and dependency order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/fse.h"
#include "fse_plan.h"
#include "fse_runtime.h"

namespace fse {


static double steady_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t ticket;
    fse_image_t image, out;
    fse_mask_t mask;
    fse_params_t params;
    int64_t bytes;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int64_t n_blocks = 0;
    int state = 0;  // 0 queued, 1 running, 2 done, 3 failed
    fse_status_t status = FSE_OK;
};

// A slot: a stream, and a thread that plans and launches the groups the
// scheduler hands to it, so that the host planning of one group overlaps the
// admission and planning of others.
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done_ev = nullptr;
    std::vector<std::shared_ptr<Request>> reqs;
    int64_t bytes = 0;
    bool busy = false;      // holds a group (being planned, or launched)
    bool assigned = false;  // a group waits for the slot's thread
    bool launched = false;  // the group's launch is enqueued and done_ev recorded
    fse_params_t params{};
    std::vector<fse_image_t> images, outs;
    std::vector<fse_mask_t> masks;
    std::thread thread;
};

}  // namespace fse

struct fse_server {
    fse_serve_config_t cfg{};
    std::mutex mu;
    std::condition_variable cv;       // wakes the scheduler
    std::condition_variable done_cv;  // wakes waiters
    std::deque<std::shared_ptr<fse::Request>> queue;
    std::map<uint64_t, std::shared_ptr<fse::Request>> all;
    std::vector<fse::Slot> slots;
    int64_t bytes_in_use = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    bool stop_slots = false;
    std::condition_variable slot_cv;  // wakes the slot threads
    std::thread worker;
};

namespace fse {

// Device memory one request needs beyond its caller-owned buffers: FP64
// reconstructed values per pixel, the fine-cell owner map, block tables,
// tickets and flags (upper bounds).
static int64_t request_bytes(const fse_image_t& im, const fse_params_t& p) {
    const int64_t px = (int64_t)im.width * im.height;
    int bmin = p.classes[p.n_classes - 1].block;
    if (bmin < 1) bmin = 1;
    const int64_t cells = ((int64_t)im.width + bmin - 1) / bmin * (((int64_t)im.height + bmin - 1) / bmin);
    int64_t tiles_extra = 0;
    if (p.tiling != FSE_WHOLE) tiles_extra = px;  // overlap stripes, generous
    return (px + tiles_extra) * 8 + cells * (4 + 16 + 16 + 4 + 8);
}

// Requests can share a launch when every field that the kernels read agrees.
static bool same_params(const fse_params_t& a, const fse_params_t& b) {
    if (a.n_classes != b.n_classes || a.rho != b.rho || a.gamma != b.gamma || a.recon_weight != b.recon_weight ||
        a.precision != b.precision || a.schedule != b.schedule || a.tiling != b.tiling || a.workgroups != b.workgroups ||
        a.block_waves != b.block_waves || a.order != b.order)
        return false;
    for (int c = 0; c < a.n_classes; ++c)
        if (a.classes[c].block != b.classes[c].block || a.classes[c].border != b.classes[c].border ||
            a.classes[c].iters != b.classes[c].iters)
            return false;
    if (a.tiling != FSE_WHOLE && (a.n_tiles != b.n_tiles || a.overlap != b.overlap || a.align != b.align)) return false;
    return true;
}

// Marks the requests of a slot's launch finished with status st (FSE_OK:
// done; otherwise failed) and frees the slot and its share of the budget.
static void finish_slot(fse_server* S, Slot& sl, fse_status_t st) {
    const double t = steady_ms();
    for (auto& r : sl.reqs) {
        r->t_done = t;
        if (r->state == 1) {
            r->state = st == FSE_OK ? 2 : 3;
            r->status = st;
        }
    }
    S->bytes_in_use -= sl.bytes;
    sl.reqs.clear();
    sl.bytes = 0;
    sl.busy = false;
    S->done_cv.notify_all();
}

// One pass of the scheduler with S->mu held by lk: retire finished launches,
// then admit queued requests into a free slot.  Returns false once the
// server is stopping and has nothing left to run.  An exception leaves the
// server consistent: every allocation happens before the state changes.
static bool schedule_once(fse_server* S, std::unique_lock<std::mutex>& lk) {
    // retire finished launches: a launch whose dependency wait hit its time
    // limit (the launch's error word) fails its requests, as does an error
    // of the completion event itself
    bool any_running = false;
    for (auto& sl : S->slots) {
        if (!sl.busy) continue;
        if (!sl.launched) {  // still being planned by its thread
            any_running = true;
            continue;
        }
        const hipError_t q = hipEventQuery(sl.done_ev);
        if (q == hipErrorNotReady) {
            any_running = true;
            continue;
        }
        fse_status_t st = from_hip(q);
        if (st == FSE_OK) {
            int32_t err = 0;
            st = read_launch_error(sl.stream, &err);
            if (st == FSE_OK && err) st = FSE_ERR_DEVICE;
        }
        finish_slot(S, sl, st);
    }
    if (S->stop && S->queue.empty() && !any_running) return false;
    // admit: FIFO, by budget, one launch per free slot, same parameters per launch
    int free_slot = -1;
    for (size_t i = 0; i < S->slots.size(); ++i)
        if (!S->slots[i].busy) {
            free_slot = (int)i;
            break;
        }
    if (free_slot >= 0 && !S->queue.empty()) {
        std::vector<std::shared_ptr<Request>> take;
        std::vector<fse_image_t> ims, outs;
        std::vector<fse_mask_t> mks;
        int64_t bytes = 0;
        const fse_params_t p0 = S->queue.front()->params;
        for (auto& r : S->queue) {
            if (!same_params(r->params, p0)) continue;
            if (S->bytes_in_use + bytes + r->bytes > S->cfg.hbm_budget_bytes) break;
            bytes += r->bytes;
            take.push_back(r);
            ims.push_back(r->image);
            outs.push_back(r->out);
            mks.push_back(r->mask);
        }
        if (!take.empty()) {
            Slot& sl = S->slots[free_slot];
            // the group's arguments go to the slot (reserved before any state
            // changes, so that an allocation failure leaves the queue intact)
            sl.images.reserve(ims.size());
            sl.outs.reserve(outs.size());
            sl.masks.reserve(mks.size());
            // the picked requests leave the queue (in queue order; no allocation)
            size_t k = 0;
            S->queue.erase(std::remove_if(S->queue.begin(), S->queue.end(),
                                          [&](const std::shared_ptr<Request>& r) {
                                              if (k < take.size() && r == take[k]) {
                                                  ++k;
                                                  return true;
                                              }
                                              return false;
                                          }),
                           S->queue.end());
            sl.busy = true;
            sl.launched = false;
            sl.assigned = true;
            sl.reqs.swap(take);
            sl.bytes = bytes;
            sl.images.swap(ims);
            sl.outs.swap(outs);
            sl.masks.swap(mks);
            sl.params = p0;
            sl.params.trace_sel = nullptr;
            S->bytes_in_use += bytes;
            const double t = steady_ms();
            for (auto& r : sl.reqs) {
                r->t_admit = t;
                r->state = 1;
            }
            S->slot_cv.notify_all();
            return true;  // try to fill another slot at once
        }
    }
    S->cv.wait_for(lk, std::chrono::microseconds(any_running ? 100 : 2000));
    return true;
}

// A slot's thread: plans and launches each group handed to the slot on the
// slot's stream (run_batch), records the completion event, and hands the
// launch back to the scheduler.
static void slot_thread(fse_server* S, size_t idx) {
    (void)hipSetDevice(S->cfg.device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        Slot& sl = S->slots[idx];
        S->slot_cv.wait(lk, [&] { return sl.assigned || S->stop_slots; });
        if (!sl.assigned) break;
        sl.assigned = false;
        const int n = (int)sl.images.size();
        lk.unlock();
        // the slot's group is not touched by anyone else until it is launched
        fse_status_t s = abi_guard([&] {
            return run_batch(n, sl.images.data(), sl.masks.data(), &sl.params, sl.outs.data(), sl.stream);
        });
        fse_run_stats_t st{};
        fse_last_stats_nowait(&st);
        if (s == FSE_OK && hipEventRecord(sl.done_ev, sl.stream) != hipSuccess) s = FSE_ERR_DEVICE;
        lk.lock();
        const int64_t per = sl.reqs.empty() ? 0 : st.n_blocks / (int64_t)sl.reqs.size();
        for (auto& r : sl.reqs) r->n_blocks = per;
        if (s != FSE_OK)
            finish_slot(S, sl, s);
        else
            sl.launched = true;
        S->cv.notify_all();
    }
}

static void scheduler(fse_server* S) {
    (void)hipSetDevice(S->cfg.device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        try {
            if (!schedule_once(S, lk)) break;
        } catch (...) {
            // out of host memory while admitting: the request at the front of
            // the queue fails, so that the next pass makes progress
            if (!lk.owns_lock()) lk.lock();
            if (!S->queue.empty()) {
                std::shared_ptr<Request> r = S->queue.front();
                S->queue.pop_front();
                r->state = 3;
                r->status = FSE_ERR_OUT_OF_MEMORY;
                r->t_done = steady_ms();
                S->done_cv.notify_all();
            }
        }
    }
}

}  // namespace fse

using namespace fse;

extern "C" {

fse_status_t fse_serve_create(const fse_serve_config_t* cfg, fse_server_t** server) {
    return abi_guard([&]() -> fse_status_t {
        if (!cfg || !server || cfg->max_slots < 1 || cfg->max_slots > 16 || cfg->hbm_budget_bytes <= 0)
            return FSE_ERR_INVALID_ARG;
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev) return FSE_ERR_INVALID_ARG;
        // the streams are created on the server's device; the caller's current
        // device is restored on return
        int prev_dev = 0;
        (void)hipGetDevice(&prev_dev);
        struct RestoreDevice {
            int d;
            ~RestoreDevice() { (void)hipSetDevice(d); }
        } restore{prev_dev};
        // streams and events are destroyed, and the server freed, on every
        // early return (and on an exception)
        auto cleanup = [](fse_server* q) {
            for (auto& s2 : q->slots) {
                if (s2.stream) (void)hipStreamDestroy(s2.stream);
                if (s2.done_ev) (void)hipEventDestroy(s2.done_ev);
            }
            delete q;
        };
        std::unique_ptr<fse_server, decltype(cleanup)> holder(new fse_server(), cleanup);
        fse_server* S = holder.get();
        S->cfg = *cfg;
        if (hipSetDevice(cfg->device) != hipSuccess) return FSE_ERR_DEVICE;
        S->slots.resize(cfg->max_slots);
        // Slot streams with a CU mask (all CUs): such a stream is given a hardware
        // queue of its own, while plain streams share the runtime's small queue
        // pool with every other stream of the process -- two slots on one queue
        // would run their launches one after the other.
        int cus = 0;
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, cfg->device);
        std::vector<uint32_t> cu_mask((size_t)std::max(1, (cus + 31) / 32), 0xffffffffu);
        for (auto& sl : S->slots) {
            if (hipExtStreamCreateWithCUMask(&sl.stream, (uint32_t)cu_mask.size(), cu_mask.data()) != hipSuccess) {
                sl.stream = nullptr;
                (void)hipGetLastError();
                if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) sl.stream = nullptr;
            }
            if (!sl.stream || hipEventCreateWithFlags(&sl.done_ev, hipEventDisableTiming) != hipSuccess)
                return FSE_ERR_DEVICE;
        }
        // the slot threads, then the scheduler; threads already started are
        // stopped and joined if a later one cannot be started
        size_t started = 0;
        try {
            for (; started < S->slots.size(); ++started) S->slots[started].thread = std::thread(slot_thread, S, started);
            S->worker = std::thread(scheduler, S);
        } catch (...) {
            {
                std::lock_guard<std::mutex> lk(S->mu);
                S->stop_slots = true;
                S->slot_cv.notify_all();
            }
            for (size_t i = 0; i < started; ++i) S->slots[i].thread.join();
            throw;
        }
        *server = holder.release();
        return FSE_OK;
    });
}

fse_status_t fse_serve_submit(fse_server_t* S, const fse_image_t* image, const fse_mask_t* mask,
                              const fse_params_t* p, fse_image_t* out, uint64_t* ticket) {
    return abi_guard([&]() -> fse_status_t {
        if (!S || !image || !mask || !p || !out || !ticket) return FSE_ERR_INVALID_ARG;
        std::vector<ClassCfg> cls;
        fse_status_t s = check_params(p, cls);
        if (s != FSE_OK) return s;
        if (!image->data || !out->data || !mask->data || image->width < 1 || image->height < 1 ||
            mask->width != image->width || mask->height != image->height || out->width != image->width ||
            out->height != image->height || image->pitch < image->width || out->pitch < out->width ||
            mask->pitch < mask->width || out->data == image->data)
            return FSE_ERR_INVALID_ARG;
        auto r = std::make_shared<Request>();
        r->image = *image;
        r->mask = *mask;
        r->out = *out;
        r->params = *p;
        r->params.trace_sel = nullptr;
        r->bytes = request_bytes(*image, *p);
        if (r->bytes > S->cfg.hbm_budget_bytes) return FSE_ERR_BUDGET;
        r->t_submit = steady_ms();
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) return FSE_ERR_BUSY;
        r->ticket = S->next_ticket++;
        S->all[r->ticket] = r;
        try {
            S->queue.push_back(r);
        } catch (...) {
            S->all.erase(r->ticket);
            throw;
        }
        *ticket = r->ticket;
        S->cv.notify_one();
        return FSE_OK;
    });
}

static void fill_stats(const Request& r, fse_request_stats_t* st) {
    if (!st) return;
    st->t_submit_ms = r.t_submit;
    st->t_admit_ms = r.t_admit;
    st->t_done_ms = r.t_done;
    st->n_blocks = r.n_blocks;
}

fse_status_t fse_serve_poll(fse_server_t* S, uint64_t ticket, int32_t* done, fse_request_stats_t* st) {
    return abi_guard([&]() -> fse_status_t {
        if (!S || !done) return FSE_ERR_INVALID_ARG;
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->all.find(ticket);
        if (it == S->all.end()) return FSE_ERR_NOT_FOUND;
        const Request& r = *it->second;
        *done = r.state >= 2;
        fill_stats(r, st);
        return r.state == 3 ? r.status : FSE_OK;
    });
}

fse_status_t fse_serve_wait(fse_server_t* S, uint64_t ticket, int64_t timeout_us, fse_request_stats_t* st) {
    return abi_guard([&]() -> fse_status_t {
        if (!S) return FSE_ERR_INVALID_ARG;
        std::unique_lock<std::mutex> lk(S->mu);
        auto it = S->all.find(ticket);
        if (it == S->all.end()) return FSE_ERR_NOT_FOUND;
        auto r = it->second;
        auto pred = [&] { return r->state >= 2; };
        if (timeout_us < 0) {
            S->done_cv.wait(lk, pred);
        } else if (!S->done_cv.wait_for(lk, std::chrono::microseconds(timeout_us), pred)) {
            return FSE_ERR_TIMEOUT;
        }
        fill_stats(*r, st);
        const fse_status_t s = r->state == 3 ? r->status : FSE_OK;
        S->all.erase(ticket);
        return s;
    });
}

fse_status_t fse_serve_cancel(fse_server_t* S, uint64_t ticket) {
    return abi_guard([&]() -> fse_status_t {
        if (!S) return FSE_ERR_INVALID_ARG;
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->all.find(ticket);
        if (it == S->all.end()) return FSE_ERR_NOT_FOUND;
        const std::shared_ptr<Request> r = it->second;
        if (r->state != 0) return FSE_ERR_BUSY;  // admitted into a launch (or finished): it runs to the end
        S->queue.erase(std::remove(S->queue.begin(), S->queue.end(), r), S->queue.end());
        r->state = 3;
        r->status = FSE_ERR_CANCELLED;
        r->t_done = steady_ms();
        S->done_cv.notify_all();
        return FSE_OK;
    });
}

fse_status_t fse_serve_destroy(fse_server_t* S) {
    return abi_guard([&]() -> fse_status_t {
        if (!S) return FSE_ERR_INVALID_ARG;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop = true;
            S->cv.notify_all();
        }
        if (S->worker.joinable()) S->worker.join();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop_slots = true;
            S->slot_cv.notify_all();
        }
        for (auto& sl : S->slots)
            if (sl.thread.joinable()) sl.thread.join();
        int prev_dev = 0;
        (void)hipGetDevice(&prev_dev);
        (void)hipSetDevice(S->cfg.device);
        for (auto& sl : S->slots) {
            (void)hipStreamSynchronize(sl.stream);
            release_workspace(S->cfg.device, sl.stream);  // the slot's device tables and staging
            (void)hipStreamDestroy(sl.stream);
            (void)hipEventDestroy(sl.done_ev);
        }
        (void)hipSetDevice(prev_dev);
        delete S;
        return FSE_OK;
    });
}

}  // extern "C"
