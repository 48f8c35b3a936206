// fse_api.cpp -- the C ABI of libfse: argument checks, workspace, planning
// and launches.  See include/fse.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/fse.h"
#include "fse_internal.h"
#include "fse_plan.h"
#include "fse_runtime.h"

namespace fse {

thread_local fse_run_stats_t g_last_stats{};
// the workspace of this thread's last call, by registry key and generation
// (a released workspace is then recognised instead of dereferenced)
struct LastCall {
    int dev = -1;
    hipStream_t st = nullptr;
    uint64_t gen = 0;
    // a call of fse_extrapolate_noalloc: its completion event and error words
    hipEvent_t noalloc_done = nullptr;
    const int32_t* noalloc_misc = nullptr;
};
thread_local LastCall g_last;

void set_last_call_noalloc(const fse_run_stats_t& st, int dev, hipStream_t s, hipEvent_t done, const int32_t* misc) {
    g_last_stats = st;
    g_last = LastCall{dev, s, 0, done, misc};
}

static double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

fse_status_t from_hip(hipError_t e) {
    if (e == hipSuccess) return FSE_OK;
    if (e == hipErrorOutOfMemory) return FSE_ERR_OUT_OF_MEMORY;
    return FSE_ERR_DEVICE;
}

hipError_t DevBuf::ensure(size_t n, std::vector<void*>& retired) {
    if (n <= cap) return hipSuccess;
    if (p) {
        retired.push_back(p);
        p = nullptr;
        cap = 0;
    }
    size_t want = std::max<size_t>(n, 256);
    want = want + want / 4;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        p = nullptr;
        return e;
    }
    cap = want;
    return hipSuccess;
}

hipError_t Arena::take(DevBuf& b, size_t n) {
    const size_t want = (std::max<size_t>(n, 1) + 255) & ~(size_t)255;
    if (!dev || used > dev_cap || want > dev_cap - used) return hipErrorOutOfMemory;
    b.p = dev + used;
    b.cap = want;
    used += want;
    return hipSuccess;
}

void DevBuf::release() {
    if (p) hipFree(p);
    p = nullptr;
    cap = 0;
}

// ---------------------------------------------------------------------------
// workspaces: one per (device, stream); calls on one stream are serialised
// ---------------------------------------------------------------------------
// Lock order: the registry mutex, then a workspace's mutex.
static std::mutex g_ws_mu;
static std::map<std::pair<int, hipStream_t>, std::unique_ptr<Workspace>> g_ws;
static uint64_t g_ws_gen = 0;  // under g_ws_mu

Workspace* workspace_for(hipStream_t st, std::unique_lock<std::mutex>& lk) {
    int dev = 0;
    hipGetDevice(&dev);
    std::lock_guard<std::mutex> rl(g_ws_mu);
    auto& slot = g_ws[{dev, st}];
    if (!slot) {
        slot.reset(new Workspace());
        slot->gen = ++g_ws_gen;
    }
    lk = std::unique_lock<std::mutex>(slot->mu);
    return slot.get();
}

fse_status_t read_launch_error(hipStream_t st, int32_t* error) {
    int dev = 0;
    hipGetDevice(&dev);
    *error = 0;
    std::lock_guard<std::mutex> rl(g_ws_mu);
    auto it = g_ws.find({dev, st});
    if (it == g_ws.end()) return FSE_OK;
    Workspace& ws = *it->second;
    std::lock_guard<std::mutex> wl(ws.mu);
    if (!ws.misc.p) return FSE_OK;
    // through the launch's own stream (idle by now): a copy on the null
    // stream would also wait for the other streams of the device
    int32_t w = 0;
    hipError_t e = hipMemcpyAsync(&w, ws.misc.p, sizeof(w), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return from_hip(e);
    *error = w;
    return FSE_OK;
}

void release_workspace(int dev, hipStream_t st) {
    std::lock_guard<std::mutex> rl(g_ws_mu);
    auto it = g_ws.find({dev, st});
    if (it == g_ws.end()) return;
    {
        std::lock_guard<std::mutex> wl(it->second->mu);
        hipStreamSynchronize(st);
        it->second->free_all();
    }
    g_ws.erase(it);
}

void release_all_workspaces() {
    std::lock_guard<std::mutex> rl(g_ws_mu);
    for (auto& kv : g_ws) {
        std::lock_guard<std::mutex> wl(kv.second->mu);
        hipStreamSynchronize(kv.first.second);
        kv.second->free_all();
    }
    g_ws.clear();
}

void Workspace::free_all() {
    for (DevBuf* b : {&recon, &owner, &desc, &lbox, &done, &tickets, &jobs, &misc, &tabs}) b->release();
    for (void* q : retired_dev) hipFree(q);
    for (void* q : retired_host) hipHostFree(q);
    retired_dev.clear();
    retired_host.clear();
    tab_key.clear();
    if (host_mask) hipHostFree(host_mask);
    if (stage) hipHostFree(stage);
    stage = nullptr;
    stage_cap = 0;
    host_mask = nullptr;
    host_mask_cap = 0;
    if (ev0) hipEventDestroy(ev0);
    if (ev1) hipEventDestroy(ev1);
    ev0 = ev1 = nullptr;
    timed = false;
    std::deque<RegionPlan>().swap(plans);
    std::vector<PlanScratch>().swap(plan_scratch);
}

// ---------------------------------------------------------------------------
// parameter checks
// ---------------------------------------------------------------------------
fse_status_t check_params(const fse_params_t* p, std::vector<ClassCfg>& cls) {
    if (!p) return FSE_ERR_INVALID_ARG;
    if (p->n_classes < 1 || p->n_classes > FSE_MAX_CLASSES) return FSE_ERR_INVALID_ARG;
    if (!(p->rho > 0.0 && p->rho <= 1.0)) return FSE_ERR_INVALID_ARG;
    if (!(p->gamma > 0.0 && p->gamma < 2.0)) return FSE_ERR_INVALID_ARG;
    if (!(p->recon_weight > 0.0 && p->recon_weight <= 1.0)) return FSE_ERR_INVALID_ARG;
    if (p->precision != FSE_PREC_F64 && p->precision != FSE_PREC_F32 && p->precision != FSE_PREC_BF16X3)
        return FSE_ERR_INVALID_ARG;
    if (p->schedule < FSE_SCHED_PERSISTENT || p->schedule > FSE_SCHED_PER_BLOCK) return FSE_ERR_INVALID_ARG;
    if (p->tiling != FSE_WHOLE && p->tiling != FSE_TILED && p->tiling != FSE_TILED_VERTICAL)
        return FSE_ERR_INVALID_ARG;
    if (p->order != FSE_ORDER_RASTER && p->order != FSE_ORDER_OPTIMIZED) return FSE_ERR_INVALID_ARG;
    cls.clear();
    for (int c = 0; c < p->n_classes; ++c) {
        const fse_class_t& k = p->classes[c];
        if (k.block < 1 || k.border < 0 || k.iters < 0 || k.iters > 256) return FSE_ERR_INVALID_ARG;
        const int M = k.block + 2 * k.border;
        if (M != 32 && M != 64) return FSE_ERR_UNSUPPORTED;
        if (k.block > 16 || (k.block & (k.block - 1)) != 0) return FSE_ERR_UNSUPPORTED;
        cls.push_back({k.block, k.border, k.iters, M});
    }
    for (int c = 0; c + 1 < p->n_classes; ++c)
        if (cls[c].B <= cls[c + 1].B || cls[c].B % cls[c + 1].B) return FSE_ERR_INVALID_ARG;
    if (p->tiling != FSE_WHOLE) {
        if (p->n_tiles < 1 || p->overlap < 0 || p->align < 1) return FSE_ERR_INVALID_ARG;
        if (p->align % cls.back().B != 0) return FSE_ERR_INVALID_ARG;
        if (p->align % cls.front().B != 0) return FSE_ERR_INVALID_ARG;
    }
    if (p->block_waves != 0 && p->block_waves != 1 && p->block_waves != 2 && p->block_waves != 4)
        return FSE_ERR_INVALID_ARG;
    if (p->trace_sel) {
        int kmax = 0;
        for (auto& c : cls) kmax = std::max(kmax, c.K);
        if (p->trace_stride < kmax || p->trace_stride < 1 || p->trace_capacity < 0) return FSE_ERR_INVALID_ARG;
    }
    return FSE_OK;
}

static fse_status_t check_image(const fse_image_t* im) {
    if (!im || !im->data || im->width < 1 || im->height < 1 || im->pitch < im->width) return FSE_ERR_INVALID_ARG;
    return FSE_OK;
}

// ---------------------------------------------------------------------------
// device tables: rho^dist per class, twiddles
// ---------------------------------------------------------------------------
static fse_status_t upload_tables(Workspace& ws, const std::vector<ClassCfg>& cls, double rho, hipStream_t st,
                                  LaunchArgs& a) {
    std::vector<double> key{rho};
    for (auto& c : cls) key.insert(key.end(), {(double)c.B, (double)c.b});
    size_t total = 64 + 128;
    for (auto& c : cls) total += (size_t)c.M * c.M;
    if (ws.tab_key != key) {
        std::vector<double> h(total);
        for (int p = 0; p < 32; ++p) {
            h[p] = std::cos(2.0 * M_PI * p / 32.0);
            h[32 + p] = std::sin(2.0 * M_PI * p / 32.0);
        }
        for (int p = 0; p < 64; ++p) {
            h[64 + p] = std::cos(2.0 * M_PI * p / 64.0);
            h[128 + p] = std::sin(2.0 * M_PI * p / 64.0);
        }
        size_t off = 192;
        for (auto& c : cls) {
            const double ctr = 0.5 * (c.M - 1);
            for (int m = 0; m < c.M; ++m)
                for (int n = 0; n < c.M; ++n)
                    h[off + m * c.M + n] = std::pow(rho, std::sqrt((m - ctr) * (m - ctr) + (n - ctr) * (n - ctr)));
            off += (size_t)c.M * c.M;
        }
        hipError_t e = ws.grow(ws.tabs, total * sizeof(double));
        if (e != hipSuccess) return from_hip(e);
        e = hipMemcpyAsync(ws.tabs.p, h.data(), total * sizeof(double), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return from_hip(e);
        ws.tab_key = key;
    }
    const double* base = (const double*)ws.tabs.p;
    a.tw32 = base;
    a.tw64 = base + 64;
    size_t off = 192;
    for (size_t c = 0; c < cls.size(); ++c) {
        a.cls[c].B = cls[c].B;
        a.cls[c].b = cls[c].b;
        a.cls[c].M = cls[c].M;
        a.cls[c].K = cls[c].K;
        a.cls[c].wtab = base + off;
        off += (size_t)cls[c].M * cls[c].M;
    }
    a.n_classes = (int)cls.size();
    return FSE_OK;
}

// ---------------------------------------------------------------------------
// host parallelism for planning: fn(i) for i in [0, n) over up to 16 threads
// ---------------------------------------------------------------------------
template <class F>
static void parallel_for(size_t n, F fn) {
    const size_t hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t nt = std::min<size_t>({n, hw, (size_t)16});
    if (nt <= 1) {
        for (size_t i = 0; i < n; ++i) fn(i);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(nt);
    for (size_t k = 0; k < nt; ++k)
        th.emplace_back([&, k] {
            for (size_t i = k; i < n; i += nt) fn(i);
        });
    for (auto& x : th) x.join();
}

// ---------------------------------------------------------------------------
// the extrapolation call
// ---------------------------------------------------------------------------
struct HostJob {
    int img;             // index of the image in the batch
    int ox, oy, W, H;    // region
    int cx0, cy0, cx1, cy1;
    RegionPlan* plan;  // kept in the workspace between calls (memory reuse)
};

static fse_status_t check_batch(int n, const fse_image_t* images, const fse_mask_t* masks, const fse_params_t* p,
                                const fse_image_t* outs, std::vector<ClassCfg>& cls) {
    if (n < 1 || !images || !masks || !outs) return FSE_ERR_INVALID_ARG;
    fse_status_t s = check_params(p, cls);
    if (s != FSE_OK) return s;
    for (int i = 0; i < n; ++i) {
        if (check_image(&images[i]) != FSE_OK || check_image(&outs[i]) != FSE_OK) return FSE_ERR_INVALID_ARG;
        const fse_mask_t& m = masks[i];
        if (!m.data || m.width != images[i].width || m.height != images[i].height || m.pitch < m.width)
            return FSE_ERR_INVALID_ARG;
        if (outs[i].width != images[i].width || outs[i].height != images[i].height) return FSE_ERR_INVALID_ARG;
        if (outs[i].data == images[i].data) return FSE_ERR_INVALID_ARG;
    }
    return FSE_OK;
}

fse_status_t run_batch(int n, const fse_image_t* images, const fse_mask_t* masks, const fse_params_t* p,
                       fse_image_t* outs, hipStream_t st) {
    std::vector<ClassCfg> cls;
    fse_status_t s = check_batch(n, images, masks, p, outs, cls);
    if (s != FSE_OK) return s;
    std::unique_lock<std::mutex> lk;
    Workspace& ws = *workspace_for(st, lk);
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return from_hip(e);
    Prepared P;
    if ((s = prepare_batch(ws, n, images, masks, p, outs, cls, st, P)) != FSE_OK) return s;
    if ((s = launch_prepared(ws, P, st, true)) != FSE_OK) return s;
    ws.last_stream = st;
    g_last_stats = P.stats;
    int dev = 0;
    hipGetDevice(&dev);
    g_last = LastCall{dev, st, ws.gen};
    return FSE_OK;
}

// Bound of every dependency wait, in s_memrealtime ticks (100 MHz): 5 s, or
// FSE_WAIT_LIMIT_US microseconds from the environment (read when a launch is
// prepared).  A wait that reaches it sets the launch's error flag and goes
// on, so a lost wake-up ends as an error instead of a hang.
static int64_t wait_limit_ticks() {
    int64_t us = 5000000;
    if (const char* e = std::getenv("FSE_WAIT_LIMIT_US")) {
        char* end = nullptr;
        const long long v = std::strtoll(e, &end, 10);
        if (end != e && v >= 0) us = v;
    }
    return us * 100;
}

fse_status_t prepare_batch(Workspace& ws, int n, const fse_image_t* images, const fse_mask_t* masks,
                           const fse_params_t* p, const fse_image_t* outs, const std::vector<ClassCfg>& cls,
                           hipStream_t st, Prepared& P) {
    fse_run_stats_t stats{};
    fse_status_t s = FSE_OK;
    hipError_t e = hipSuccess;
    const double t0 = now_ms();
    if (ws.arena) {
        // every call carves its buffers afresh; the tables are uploaded again
        ws.arena->used = 0;
        for (DevBuf* b : {&ws.recon, &ws.owner, &ws.desc, &ws.lbox, &ws.done, &ws.tickets, &ws.jobs, &ws.misc,
                          &ws.tabs})
            *b = DevBuf{};
        ws.tab_key.clear();
        ws.host_mask = ws.arena->host_mask;
        ws.host_mask_cap = ws.arena->host_mask_cap;
        ws.stage = ws.arena->host_stage;
        ws.stage_cap = ws.arena->host_stage_cap;
    }
    // ---- masks to the host, regions, plans ---------------------------------
    std::vector<HostJob> jobs;
    std::vector<size_t> moff(n + 1, 0);
    for (int i = 0; i < n; ++i) moff[i + 1] = moff[i] + (size_t)images[i].width * images[i].height;
    if (ws.host_mask_cap < moff[n]) {
        if (ws.arena) return FSE_ERR_BUDGET;
        // pinned memory grows with headroom; the old block is retired, not
        // freed (hipHostFree waits for the whole device)
        if (ws.host_mask) ws.retired_host.push_back(ws.host_mask);
        ws.host_mask = nullptr;
        ws.host_mask_cap = 0;
        const size_t want = moff[n] + moff[n] / 4;
        if ((e = hipHostMalloc((void**)&ws.host_mask, want, hipHostMallocDefault)) != hipSuccess)
            return from_hip(e);
        ws.host_mask_cap = want;
    }
    for (int i = 0; i < n; ++i) {
        const int W = images[i].width, H = images[i].height;
        e = hipMemcpy2DAsync(ws.host_mask + moff[i], W, masks[i].data, masks[i].pitch, W, H, hipMemcpyDeviceToHost,
                             st);
        if (e != hipSuccess) return from_hip(e);
    }
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return from_hip(e);
    for (int i = 0; i < n; ++i) {
        const int W = images[i].width, H = images[i].height;
        if (p->tiling == FSE_WHOLE) {
            HostJob J{i, 0, 0, W, H, 0, 0, W, H, nullptr};
            jobs.push_back(std::move(J));
        } else {
            std::vector<fse_tile_t> tiles(p->n_tiles);
            s = p->tiling == FSE_TILED_VERTICAL
                    ? fse_plan_tiles_vertical(W, H, p->n_tiles, p->overlap, p->align, tiles.data())
                    : fse_plan_tiles(W, H, p->n_tiles, p->overlap, p->align, tiles.data());
            if (s != FSE_OK) return s;
            for (auto& T : tiles) {
                if (T.w <= 0 || T.h <= 0) continue;
                HostJob J{i, T.ox, T.oy, T.ow, T.oh, T.x - T.ox, T.y - T.oy, T.x - T.ox + T.w, T.y - T.oy + T.h, nullptr};
                jobs.push_back(std::move(J));
            }
        }
    }
    int reach = 0;  // largest support border: the reach of the kernel's dependency scan
    for (auto& c : cls) reach = std::max(reach, c.b);
    // plans and planning scratch live in the workspace (memory reused)
    while (ws.plans.size() < jobs.size()) ws.plans.emplace_back();
    if (ws.plan_scratch.size() < jobs.size()) ws.plan_scratch.resize(jobs.size());
    for (size_t j = 0; j < jobs.size(); ++j) jobs[j].plan = &ws.plans[j];
    std::vector<uint8_t> plan_ok(jobs.size(), 1);
    // host threads for the optimised order's pair lists within one job: the
    // jobs already run in parallel, so each gets its share of the threads
    const int order_threads =
        (int)std::max<size_t>(1, std::min<size_t>(16, std::max(1u, std::thread::hardware_concurrency())) / jobs.size());
    parallel_for(jobs.size(), [&](size_t j) {
        HostJob& J = jobs[j];
        const uint8_t* mk = ws.host_mask + moff[J.img] + (size_t)J.oy * images[J.img].width + J.ox;
        plan_ok[j] = plan_region(mk, images[J.img].width, J.W, J.H, cls, *J.plan, ws.plan_scratch[j]);
        if (plan_ok[j] && p->order == FSE_ORDER_OPTIMIZED) {
            // blocks renumbered in the optimised order; levels (and the
            // wavefront keys) over exactly the waits of that order
            plan_priority_order(*J.plan, mk, images[J.img].width, cls, p->rho, p->recon_weight,
                                ws.plan_scratch[j].order, order_threads);
        } else if (plan_ok[j] && p->schedule == FSE_SCHED_PERSISTENT) {
            plan_levels(*J.plan, cls, reach, ws.plan_scratch[j].cell_level);
        }
    });
    for (size_t j = 0; j < jobs.size(); ++j) {
        if (!plan_ok[j]) return FSE_ERR_INVALID_ARG;
        stats.n_blocks += (int64_t)(jobs[j].plan->desc.size() / 4);
    }
    for (auto& J : jobs) stats.n_lost_pixels += J.plan->lost_pixels;
    stats.n_jobs = (int64_t)jobs.size();

    // ---- ticket order: a counting sort of all blocks of all jobs -------------
    // The persistent schedule orders by dependency level (a topological order
    // that keeps ready blocks ahead of blocks deep in a chain); the other
    // schedules by wavefront key (the wavefront schedule launches one key at a
    // time).  Within a bucket: job, then raster order.  Per-job histograms and
    // the placement run in parallel; the tickets go straight into the pinned
    // staging buffer below.
    const bool by_level = p->schedule == FSE_SCHED_PERSISTENT;
    const int64_t ntk = stats.n_blocks;
    const size_t nj = jobs.size();
    auto sort_key = [&](size_t j) -> const std::vector<int32_t>& {
        return by_level ? jobs[j].plan->level : jobs[j].plan->key;
    };
    std::vector<int32_t> job_max(nj, 0);
    parallel_for(nj, [&](size_t j) {
        int m = 0;
        for (int k : sort_key(j)) m = std::max(m, k);
        job_max[j] = m;
    });
    int max_key = 0;
    for (int m : job_max) max_key = std::max(max_key, m);
    const size_t nb_keys = (size_t)max_key + 1;
    std::vector<int32_t> off(nj * nb_keys, 0);  // per job: histogram, then bucket offsets
    parallel_for(nj, [&](size_t j) {
        int32_t* h = &off[j * nb_keys];
        for (int k : sort_key(j)) h[k]++;
    });
    std::vector<int32_t> kstart(nb_keys + 1, 0);
    int nkeys = 0;
    {
        int64_t run = 0;
        for (size_t k = 0; k < nb_keys; ++k) {
            kstart[k] = (int32_t)run;
            const int64_t before = run;
            for (size_t j = 0; j < nj; ++j) {
                const int32_t c = off[j * nb_keys + k];
                off[j * nb_keys + k] = (int32_t)run;
                run += c;
            }
            nkeys += run > before;
        }
        kstart[nb_keys] = (int32_t)run;
    }
    stats.wavefront_keys = nkeys;  // distinct levels (persistent) or keys (other schedules)
    const int n_levels = nkeys;

    // ---- device buffers -----------------------------------------------------
    size_t n_pix = 0, n_cells = 0, n_blk = 0;
    for (auto& J : jobs) {
        n_pix += (size_t)J.W * J.H;
        n_cells += J.plan->owner.size();
        n_blk += J.plan->desc.size() / 4;
    }
    // (from the arena, a buffer that does not fit is a budget error: the
    // arena's size is fixed)
    auto grow = [&](DevBuf& b, size_t bytes) -> fse_status_t {
        const hipError_t ge = ws.grow(b, bytes);
        return ge == hipSuccess ? FSE_OK : ws.arena ? FSE_ERR_BUDGET : from_hip(ge);
    };
    if ((s = grow(ws.recon, n_pix * sizeof(double))) != FSE_OK) return s;
    if ((s = grow(ws.owner, std::max<size_t>(n_cells, 1) * 4)) != FSE_OK) return s;
    if ((s = grow(ws.desc, std::max<size_t>(n_blk, 1) * 16)) != FSE_OK) return s;
    if ((s = grow(ws.lbox, std::max<size_t>(n_blk, 1) * 16)) != FSE_OK) return s;
    if ((s = grow(ws.done, std::max<size_t>(n_blk, 1) * 4)) != FSE_OK) return s;
    if ((s = grow(ws.tickets, (size_t)std::max<int64_t>(ntk, 1) * 8)) != FSE_OK) return s;
    if ((s = grow(ws.jobs, jobs.size() * sizeof(JobDev))) != FSE_OK) return s;
    if ((s = grow(ws.misc, 64)) != FSE_OK) return s;
    if (ws.arena) {
        // the tables (twiddles and rho^dist per class) take the arena's next range
        size_t tab = 64 + 128;
        for (auto& c : cls) tab += (size_t)c.M * c.M;
        const size_t tab_bytes = (tab * sizeof(double) + 255) & ~(size_t)255;
        if (ws.arena->used > ws.arena->dev_cap || tab_bytes > ws.arena->dev_cap - ws.arena->used)
            return FSE_ERR_BUDGET;
    }

    // host images of the tables in pinned staging memory, one upload each
    const size_t b_owner = std::max<size_t>(n_cells, 1) * 4, b_desc = std::max<size_t>(n_blk, 1) * 16,
                 b_tk = std::max<int64_t>(ntk, 1) * 8, b_jobs = jobs.size() * sizeof(JobDev);
    const size_t o_owner = 0, o_desc = o_owner + ((b_owner + 255) & ~(size_t)255),
                 o_lbox = o_desc + ((b_desc + 255) & ~(size_t)255), o_tk = o_lbox + ((b_desc + 255) & ~(size_t)255),
                 o_jobs = o_tk + ((b_tk + 255) & ~(size_t)255), stage_bytes = o_jobs + b_jobs + 256;
    if (ws.stage_cap < stage_bytes) {
        if (ws.arena) return FSE_ERR_BUDGET;
        if (ws.stage) ws.retired_host.push_back(ws.stage);
        ws.stage = nullptr;
        ws.stage_cap = 0;
        const size_t want = stage_bytes + stage_bytes / 4;
        if ((e = hipHostMalloc((void**)&ws.stage, want, hipHostMallocDefault)) != hipSuccess) return from_hip(e);
        ws.stage_cap = want;
    }
    int32_t* h_owner = (int32_t*)(ws.stage + o_owner);
    int32_t* h_desc = (int32_t*)(ws.stage + o_desc);
    int32_t* h_lbox = (int32_t*)(ws.stage + o_lbox);
    JobDev* h_jobs = (JobDev*)(ws.stage + o_jobs);
    {
        int32_t* tk = (int32_t*)(ws.stage + o_tk);
        parallel_for(nj, [&](size_t j) {
            int32_t* o = &off[j * nb_keys];
            const std::vector<int32_t>& sk = sort_key(j);
            for (size_t b = 0; b < sk.size(); ++b) {
                const int32_t pos = o[sk[b]]++;
                tk[2 * pos] = (int32_t)j;
                tk[2 * pos + 1] = (int32_t)b;
            }
        });
    }
    std::vector<size_t> off_pix(jobs.size() + 1, 0), off_cell(jobs.size() + 1, 0), off_blk(jobs.size() + 1, 0);
    for (size_t j = 0; j < jobs.size(); ++j) {
        off_pix[j + 1] = off_pix[j] + (size_t)jobs[j].W * jobs[j].H;
        off_cell[j + 1] = off_cell[j] + jobs[j].plan->owner.size();
        off_blk[j + 1] = off_blk[j] + jobs[j].plan->desc.size() / 4;
    }
    parallel_for(jobs.size(), [&](size_t j) {
        const HostJob& J = jobs[j];
        const size_t nb = J.plan->desc.size() / 4;
        const size_t o_pix = off_pix[j], o_cell = off_cell[j], o_blk = off_blk[j];
        std::copy(J.plan->owner.begin(), J.plan->owner.end(), h_owner + o_cell);
        std::copy(J.plan->desc.begin(), J.plan->desc.end(), h_desc + 4 * o_blk);
        std::copy(J.plan->lbox.begin(), J.plan->lbox.end(), h_lbox + 4 * o_blk);
        JobDev D{};
        D.img = images[J.img].data;
        D.mask = masks[J.img].data;
        D.out = outs[J.img].data;
        D.img_pitch = images[J.img].pitch;
        D.mask_pitch = masks[J.img].pitch;
        D.out_pitch = outs[J.img].pitch;
        D.recon = (double*)ws.recon.p + o_pix;
        D.W = J.W;
        D.H = J.H;
        D.ox = J.ox;
        D.oy = J.oy;
        D.cx0 = J.cx0;
        D.cy0 = J.cy0;
        D.cx1 = J.cx1;
        D.cy1 = J.cy1;
        D.fw = J.plan->fw;
        D.fh = J.plan->fh;
        D.owner = (const int32_t*)ws.owner.p + o_cell;
        D.desc = (const int4*)ws.desc.p + o_blk;
        D.lbox = (const int4*)ws.lbox.p + o_blk;
        D.done = (int32_t*)ws.done.p + o_blk;
        D.n_blocks = (int32_t)nb;
        const bool tr = p->trace_sel && p->tiling == FSE_WHOLE && n == 1;
        D.trace = tr ? p->trace_sel : nullptr;
        D.trace_stride = tr ? p->trace_stride : 0;
        D.trace_cap = tr ? p->trace_capacity : 0;
        h_jobs[j] = D;
    });
    auto up = [&](DevBuf& b, const void* h, size_t bytes) {
        return bytes ? hipMemcpyAsync(b.p, h, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
    };
    if ((e = up(ws.owner, h_owner, n_cells * 4)) != hipSuccess) return from_hip(e);
    if ((e = up(ws.desc, h_desc, n_blk * 16)) != hipSuccess) return from_hip(e);
    if ((e = up(ws.lbox, h_lbox, n_blk * 16)) != hipSuccess) return from_hip(e);
    if ((e = up(ws.tickets, ws.stage + o_tk, (size_t)ntk * 8)) != hipSuccess) return from_hip(e);
    if ((e = up(ws.jobs, h_jobs, jobs.size() * sizeof(JobDev))) != hipSuccess) return from_hip(e);

    LaunchArgs a{};
    if ((s = upload_tables(ws, cls, p->rho, st, a)) != FSE_OK) return s;
    a.jobs = (const JobDev*)ws.jobs.p;
    a.tickets = (const int2*)ws.tickets.p;
    a.n_tickets = (int32_t)ntk;
    int32_t* misc = (int32_t*)ws.misc.p;
    a.error = misc;
    a.degenerate = (int64_t*)(misc + 2);
    a.Bmin = cls.back().B;
    a.reach = reach;
    a.gamma = p->gamma;
    a.delta = p->recon_weight;
    a.wait_limit = wait_limit_ticks();
    stats.host_plan_ms = now_ms() - t0;

    int max_w = 1, max_h = 1;
    for (auto& J : jobs) {
        max_w = std::max(max_w, J.W);
        max_h = std::max(max_h, J.H);
    }
    a.counter = misc + 1;
    bool wide = false;
    for (auto& c : cls) wide |= (c.M == 64);
    const int nw = wide ? kWideWaves : (p->block_waves > 0 ? p->block_waves : 4);
    // Automatic grid: about twice the average number of blocks per dependency
    // level (per wavefront key for the other schedules).  A dependency chain
    // runs fastest when its blocks do not
    // share SIMDs with blocks that cannot start yet, so a grid much larger than
    // the available parallelism only slows the chain.
    int grid = p->workgroups;
    if (grid <= 0) {
        const int64_t par = (ntk + std::max(1, n_levels) - 1) / std::max(1, n_levels);
        const int64_t want = std::max<int64_t>(64, ((2 * par + 63) / 64) * 64);
        grid = (int)std::min<int64_t>(want, persistent_grid(nw, p->precision, wide));
    }
    grid = (int)std::max<int64_t>(1, std::min<int64_t>(grid, ntk));
    if (p->schedule == FSE_SCHED_PER_BLOCK && ntk > 0) {
        // plain path: one launch per block, in the processing order of each job
        std::vector<int32_t> raster(2 * ntk);
        size_t q = 0;
        for (size_t j = 0; j < jobs.size(); ++j)
            for (size_t b = 0; b < jobs[j].plan->key.size(); ++b) {
                raster[2 * q] = (int32_t)j;
                raster[2 * q + 1] = (int32_t)b;
                ++q;
            }
        std::memcpy(ws.stage + o_tk, raster.data(), (size_t)ntk * 8);
        if ((e = up(ws.tickets, ws.stage + o_tk, (size_t)ntk * 8)) != hipSuccess) return from_hip(e);
    }
    P.a = a;
    P.n_jobs = (int)jobs.size();
    P.max_w = max_w;
    P.max_h = max_h;
    P.nw = nw;
    P.wide = wide;
    P.grid = grid;
    P.precision = p->precision;
    P.schedule = p->schedule;
    P.ntk = ntk;
    P.kstart = kstart;
    P.max_key = max_key;
    P.o_jobs = o_jobs;
    P.b_jobs = jobs.size() * sizeof(JobDev);
    P.job_image.clear();
    for (auto& J : jobs) P.job_image.push_back(J.img);
    P.stats = stats;
    return FSE_OK;
}

fse_status_t launch_prepared(Workspace& ws, Prepared& P, hipStream_t st, bool timed) {
    hipError_t e = launch_init_job(P.a.jobs, P.n_jobs, P.max_w, P.max_h, P.a.counter, P.a.error, P.a.degenerate, st);
    if (e != hipSuccess) return from_hip(e);
    if (timed) {
        if (!ws.ev0) {
            if ((e = hipEventCreate(&ws.ev0)) != hipSuccess) return from_hip(e);
            if ((e = hipEventCreate(&ws.ev1)) != hipSuccess) return from_hip(e);
        }
        if ((e = hipEventRecord(ws.ev0, st)) != hipSuccess) return from_hip(e);
    }
    LaunchArgs a = P.a;
    if (P.ntk > 0) {
        if (P.schedule == FSE_SCHED_PERSISTENT) {
            e = launch_blocks_at(a, P.nw, P.precision, P.wide, P.grid, 0, st);
        } else if (P.schedule == FSE_SCHED_WAVEFRONT) {
            a.counter = nullptr;
            for (int k = 0; k <= P.max_key && e == hipSuccess; ++k) {
                const int cnt = P.kstart[k + 1] - P.kstart[k];
                if (cnt > 0) e = launch_blocks_at(a, P.nw, P.precision, P.wide, cnt, P.kstart[k], st);
            }
        } else {
            a.counter = nullptr;
            for (int64_t k = 0; k < P.ntk && e == hipSuccess; ++k)
                e = launch_blocks_at(a, P.nw, P.precision, P.wide, 1, (int)k, st);
        }
        if (e != hipSuccess) return from_hip(e);
    }
    if (timed) {
        if ((e = hipEventRecord(ws.ev1, st)) != hipSuccess) return from_hip(e);
        ws.timed = true;
    }
    return FSE_OK;
}

void fse_last_stats_nowait(fse_run_stats_t* st) { *st = g_last_stats; }

}  // namespace fse

using namespace fse;

extern "C" {

const char* fse_status_string(fse_status_t s) {
    switch (s) {
        case FSE_OK: return "ok";
        case FSE_ERR_INVALID_ARG: return "invalid argument";
        case FSE_ERR_UNSUPPORTED: return "unsupported configuration";
        case FSE_ERR_BUDGET: return "request exceeds the memory budget";
        case FSE_ERR_OUT_OF_MEMORY: return "out of device memory";
        case FSE_ERR_DEVICE: return "device error";
        case FSE_ERR_TIMEOUT: return "timed out";
        case FSE_ERR_NOT_FOUND: return "unknown ticket";
        case FSE_ERR_BUSY: return "busy";
        case FSE_ERR_CANCELLED: return "cancelled";
        default: return "unknown status";
    }
}

fse_status_t fse_params_default(fse_params_t* p) {
    return abi_guard([&]() -> fse_status_t {
        if (!p) return FSE_ERR_INVALID_ARG;
        std::memset(p, 0, sizeof(*p));
        p->n_classes = 1;
        p->classes[0] = {4, 14, 100};
        p->rho = 0.8;
        p->gamma = 0.5;
        p->recon_weight = 0.5;
        p->precision = FSE_PREC_F64;
        p->schedule = FSE_SCHED_PERSISTENT;
        p->tiling = FSE_WHOLE;
        p->n_tiles = 1;
        p->overlap = 32;
        p->align = 16;
        return FSE_OK;
    });
}

}  // extern "C"

// Core tiles of a tiling, interior edges moved down to multiples of align,
// grown by the stripe d and clipped to the image.
static fse_status_t tiles_with_stripe(int32_t W, int32_t H, int32_t N, int32_t d, int32_t align, bool vertical,
                                      fse_tile_t* tiles) {
    if (W < 1 || H < 1 || N < 1 || d < 0 || align < 1 || !tiles) return FSE_ERR_INVALID_ARG;
    if ((int64_t)N > (int64_t)W * H) return FSE_ERR_INVALID_ARG;
    std::vector<int32_t> t;
    if (!(vertical ? vertical_tiling(W, H, N, t) : compact_tiling(W, H, N, t))) return FSE_ERR_INVALID_ARG;
    for (int i = 0; i < N; ++i) {
        int x = t[4 * i], y = t[4 * i + 1];
        int x1 = x + t[4 * i + 2], y1 = y + t[4 * i + 3];
        if (align > 1) {
            x = x / align * align;
            y = y / align * align;
            x1 = (x1 == W) ? W : x1 / align * align;
            y1 = (y1 == H) ? H : y1 / align * align;
        }
        x1 = std::min(x1, W);
        y1 = std::min(y1, H);
        x = std::min(x, x1);
        y = std::min(y, y1);
        fse_tile_t& T = tiles[i];
        T.x = x;
        T.y = y;
        T.w = x1 - x;
        T.h = y1 - y;
        T.ox = std::max(0, x - d);
        T.oy = std::max(0, y - d);
        T.ow = std::max(0, std::min(W, x1 + d) - T.ox);
        T.oh = std::max(0, std::min(H, y1 + d) - T.oy);
    }
    return FSE_OK;
}

extern "C" {

fse_status_t fse_plan_tiles(int32_t W, int32_t H, int32_t N, int32_t d, int32_t align, fse_tile_t* tiles) {
    return abi_guard([&]() -> fse_status_t {
        return tiles_with_stripe(W, H, N, d, align, false, tiles);
    });
}

fse_status_t fse_plan_tiles_vertical(int32_t W, int32_t H, int32_t N, int32_t d, int32_t align,
                                     fse_tile_t* tiles) {
    return abi_guard([&]() -> fse_status_t {
        return tiles_with_stripe(W, H, N, d, align, true, tiles);
    });
}

fse_status_t fse_extrapolate(const fse_image_t* image, const fse_mask_t* mask, const fse_params_t* p,
                             fse_image_t* out, void* stream) {
    return abi_guard([&]() -> fse_status_t {
        if (!image || !mask || !out) return FSE_ERR_INVALID_ARG;
        return run_batch(1, image, mask, p, out, (hipStream_t)stream);
    });
}

fse_status_t fse_extrapolate_batch(int32_t n, const fse_image_t* images, const fse_mask_t* masks,
                                   const fse_params_t* p, fse_image_t* outs, void* stream) {
    return abi_guard([&]() -> fse_status_t {
        return run_batch(n, images, masks, p, outs, (hipStream_t)stream);
    });
}

fse_status_t fse_last_stats(fse_run_stats_t* st) {
    return abi_guard([&]() -> fse_status_t {
        if (!st) return FSE_ERR_INVALID_ARG;
        // the last call's workspace, if it still exists (fse_release frees it)
        Workspace* ws = nullptr;
        std::unique_lock<std::mutex> lk;
        if (g_last.gen) {
            std::lock_guard<std::mutex> rl(g_ws_mu);
            auto it = g_ws.find({g_last.dev, g_last.st});
            if (it != g_ws.end() && it->second->gen == g_last.gen) {
                ws = it->second.get();
                lk = std::unique_lock<std::mutex>(ws->mu);
            }
        }
        if (g_last.noalloc_done) {
            // the no-allocation entry point: its error words sit in the scratch
            // (until the next such call on that device)
            hipError_t e = hipEventSynchronize(g_last.noalloc_done);
            if (e != hipSuccess) return from_hip(e);
            int32_t misc[4] = {0, 0, 0, 0};
            if (hipMemcpy(misc, g_last.noalloc_misc, sizeof(misc), hipMemcpyDeviceToHost) == hipSuccess) {
                g_last_stats.device_error = misc[0];
                int64_t deg = 0;
                std::memcpy(&deg, misc + 2, sizeof(deg));
                g_last_stats.n_degenerate = deg;
            }
        }
        if (ws) {
            hipError_t e = hipStreamSynchronize(ws->last_stream);
            if (e != hipSuccess) return from_hip(e);
            if (ws->timed) {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, ws->ev0, ws->ev1) == hipSuccess) g_last_stats.kernel_ms = ms;
            }
            int32_t misc[4] = {0, 0, 0, 0};
            if (ws->misc.p && hipMemcpy(misc, ws->misc.p, sizeof(misc), hipMemcpyDeviceToHost) == hipSuccess) {
                g_last_stats.device_error = misc[0];
                int64_t deg = 0;
                std::memcpy(&deg, misc + 2, sizeof(deg));
                g_last_stats.n_degenerate = deg;
            }
        }
        *st = g_last_stats;
        return FSE_OK;
    });
}

}  // extern "C"

namespace fse {

// ---------------------------------------------------------------------------
// schedule autotuner
// ---------------------------------------------------------------------------
namespace {

std::mutex g_tune_mu;
std::map<std::string, fse_params_t> g_tune_cache;

// Device time of one call with parameters q (the second of two runs).
fse_status_t time_call(int n, const fse_image_t* images, const fse_mask_t* masks, const fse_params_t& q,
                       fse_image_t* outs, hipStream_t st, double& ms, fse_run_stats_t* rs_out = nullptr) {
    fse_status_t s = FSE_OK;
    for (int rep = 0; rep < 2; ++rep) {
        if ((s = run_batch(n, images, masks, &q, outs, st)) != FSE_OK) return s;
        fse_run_stats_t rs{};
        if ((s = fse_last_stats(&rs)) != FSE_OK) return s;
        if (rs.device_error) return FSE_ERR_DEVICE;
        ms = rs.kernel_ms;
        if (rs_out) *rs_out = rs;
    }
    return FSE_OK;
}

// Wall time of rounds of consecutive calls spread over the streams sts
// (outputs: one set per stream), the device running several at once.
fse_status_t time_overlapped(int n, const fse_image_t* images, const fse_mask_t* masks, const fse_params_t& q,
                             const std::vector<std::vector<fse_image_t>>& outs, const std::vector<hipStream_t>& sts,
                             double& ms) {
    const int ns = (int)sts.size();
    auto round = [&](int calls) -> fse_status_t {
        for (int i = 0; i < calls; ++i) {
            std::vector<fse_image_t> o = outs[i % ns];
            fse_status_t s = run_batch(n, images, masks, &q, o.data(), sts[i % ns]);
            if (s != FSE_OK) return s;
        }
        for (hipStream_t s : sts)
            if (hipStreamSynchronize(s) != hipSuccess) return FSE_ERR_DEVICE;
        return FSE_OK;
    };
    fse_status_t s = round(ns);  // every stream's workspace, untimed
    if (s != FSE_OK) return s;
    const auto t0 = std::chrono::steady_clock::now();
    if ((s = round(2 * ns)) != FSE_OK) return s;
    ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / (2 * ns);
    for (hipStream_t st : sts) {
        int32_t err = 0;
        if ((s = read_launch_error(st, &err)) != FSE_OK) return s;
        if (err) return FSE_ERR_DEVICE;
    }
    return FSE_OK;
}

fse_status_t autotune(int32_t n, const fse_image_t* images, const fse_mask_t* masks, const fse_params_t* p,
                      fse_image_t* outs, hipStream_t st, int streams, fse_params_t* best) {
    if (!best || !p || streams < 1 || streams > 8) return FSE_ERR_INVALID_ARG;
    // the tile count is searched when the caller leaves it to the tuner
    const bool tune_tiles = p->tiling != FSE_WHOLE && p->n_tiles == 0;
    fse_params_t q0 = *p;
    q0.trace_sel = nullptr;
    if (tune_tiles) q0.n_tiles = 64;
    std::vector<ClassCfg> cls;
    fse_status_t s = check_batch(n, images, masks, &q0, outs, cls);
    if (s != FSE_OK) return s;
    if (p->schedule != FSE_SCHED_PERSISTENT) return FSE_ERR_INVALID_ARG;
    // a first call: its statistics (blocks and dependency levels of the
    // masks) key the cache together with sizes, classes and parameters
    double ms = 0;
    fse_run_stats_t rs0{};
    if ((s = time_call(n, images, masks, q0, outs, st, ms, &rs0)) != FSE_OK) return s;
    std::string key = std::to_string(streams) + "/" + std::to_string(p->block_waves) + "/" +
                      std::to_string(p->precision) + "/" +
                      std::to_string(p->tiling) + "/" + std::to_string(p->n_tiles) + "/" +
                      std::to_string(p->overlap) + "/" + std::to_string(p->align) + "/" + std::to_string(p->order) +
                      "/" + std::to_string(rs0.n_blocks) + "/" + std::to_string(rs0.wavefront_keys);
    for (auto& c : cls) key += "/" + std::to_string(c.B) + "," + std::to_string(c.b) + "," + std::to_string(c.K);
    for (int i = 0; i < n; ++i) key += "/" + std::to_string(images[i].width) + "x" + std::to_string(images[i].height);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            *best = *p;
            best->n_tiles = it->second.n_tiles;
            best->block_waves = it->second.block_waves;
            best->workgroups = it->second.workgroups;
            return FSE_OK;
        }
    }
    bool wide = false;
    for (auto& c : cls) wide |= (c.M == 64);
    // consecutive calls in flight: streams of the tuner's own, with outputs of
    // their own after the first (the caller's)
    std::vector<hipStream_t> sts{st};
    std::vector<std::vector<fse_image_t>> souts{std::vector<fse_image_t>(outs, outs + n)};
    std::vector<void*> scratch_outs;
    struct Cleanup {
        std::vector<hipStream_t>& sts;
        std::vector<void*>& bufs;
        ~Cleanup() {
            int dev = 0;
            hipGetDevice(&dev);
            for (size_t i = 1; i < sts.size(); ++i) {
                hipStreamSynchronize(sts[i]);
                release_workspace(dev, sts[i]);  // the stream's workspace, before the stream goes
                hipStreamDestroy(sts[i]);
            }
            for (void* b : bufs) hipFree(b);
        }
    } cleanup{sts, scratch_outs};
    for (int k = 1; k < streams; ++k) {
        hipStream_t x = nullptr;
        if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess) return FSE_ERR_DEVICE;
        sts.push_back(x);
        std::vector<fse_image_t> o(n);
        for (int i = 0; i < n; ++i) {
            void* b = nullptr;
            const size_t bytes = (size_t)images[i].width * images[i].height * sizeof(float);
            if (hipMalloc(&b, bytes) != hipSuccess) return FSE_ERR_OUT_OF_MEMORY;
            scratch_outs.push_back(b);
            o[i] = fse_image_t{(float*)b, images[i].width, images[i].height, images[i].width};
        }
        souts.push_back(o);
    }
    auto measure = [&](const fse_params_t& q, double& t) -> fse_status_t {
        return streams == 1 ? time_call(n, images, masks, q, outs, st, t)
                            : time_overlapped(n, images, masks, q, souts, sts, t);
    };
    fse_params_t cur = q0;
    // 1. tiles (tiled modes, when asked): N of Sec. III with the automatic grid
    if (tune_tiles) {
        double best_ms = 1e30;
        int best_n = 64;
        for (int N : {16, 32, 64, 128, 256}) {
            fse_params_t q = cur;
            q.n_tiles = N;
            q.workgroups = 0;
            double t = 0;
            if ((s = measure(q, t)) != FSE_OK) return s;
            if (t < best_ms) {
                best_ms = t;
                best_n = N;
            }
        }
        cur.n_tiles = best_n;
    }
    // 2. wave64s per block and persistent grid
    const std::vector<int> waves = wide ? std::vector<int>{0}
                                        : p->block_waves ? std::vector<int>{p->block_waves} : std::vector<int>{1, 2, 4};
    double best_ms = 1e30;
    int best_w = waves.back(), best_g = 0;
    for (int w : waves) {
        const int cap = persistent_grid(wide ? kWideWaves : w, p->precision, wide);
        // fixed sizes and fractions of the resident capacity (launches in
        // flight share it), each once
        std::vector<int> grids{0};
        for (int g : {128, 256, 384, 512, 768, 1024, cap / 4, cap / 2, 3 * cap / 4})
            if (g > 0 && g < cap && std::find(grids.begin(), grids.end(), g) == grids.end()) grids.push_back(g);
        std::sort(grids.begin() + 1, grids.end());
        grids.push_back(cap);
        for (int g : grids) {
            fse_params_t q = cur;
            q.block_waves = w;
            q.workgroups = g;
            double t = 0;
            if ((s = measure(q, t)) != FSE_OK) return s;
            if (t < best_ms) {
                best_ms = t;
                best_w = w;
                best_g = g;
            }
        }
    }
    *best = *p;
    best->n_tiles = cur.n_tiles;
    best->block_waves = best_w;
    best->workgroups = best_g;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = *best;
    return FSE_OK;
}

}  // namespace
}  // namespace fse

extern "C" {

fse_status_t fse_autotune(int32_t n, const fse_image_t* images, const fse_mask_t* masks, const fse_params_t* p,
                          fse_image_t* outs, void* stream, fse_params_t* best) {
    return abi_guard([&]() -> fse_status_t {
        return fse::autotune(n, images, masks, p, outs, (hipStream_t)stream, 1, best);
    });
}

fse_status_t fse_autotune_overlapped(int32_t n, const fse_image_t* images, const fse_mask_t* masks,
                                     const fse_params_t* p, fse_image_t* outs, int32_t streams,
                                     fse_params_t* best) {
    return abi_guard([&]() -> fse_status_t {
        if (streams < 2) return FSE_ERR_INVALID_ARG;
        return fse::autotune(n, images, masks, p, outs, nullptr, streams, best);
    });
}

fse_status_t fse_release(void) {
    return abi_guard([&]() -> fse_status_t {
        release_all_workspaces();
        return FSE_OK;
    });
}

}  // extern "C"
