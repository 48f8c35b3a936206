// fse_noalloc.hip -- fse_extrapolate_noalloc: the extrapolation call of
// fse_extrapolate with its device scratch in a fixed file-scope array, for
// callers that must not allocate device memory.
//
// The scratch holds what fse_extrapolate keeps in its workspace: the FP64
// working copy of reconstructed pixels, the fine-cell owner map, block
// descriptors and lost-pixel boxes, completion flags, the ticket list, the
// job table, the error / ticket / degenerate-count words and the twiddle and
// rho^dist tables.  The same kernels run on it (k_init_job clears the flags
// and counters on the device at every call; no memset is used).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/fse.h"
#include "fse_runtime.h"

namespace fse {

namespace {

constexpr size_t kScratchBytes = FSE_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "whole 256-byte ranges");
// Host staging: the planner's tables are uploaded from here.  A call whose
// tables fit the device scratch fits here too (the tables are part of it);
// the mask read-back needs one byte per pixel, and the FP64 working copy
// alone takes eight per pixel of the scratch.
constexpr size_t kHostStageBytes = kScratchBytes;
constexpr size_t kHostMaskBytes = kScratchBytes / 8;
constexpr int kMaxDevices = 64;

// The device scratch.  In host code `scratch` is only a stand-in for the
// symbol, not a device address: the address of each device's copy comes from
// hipGetSymbolAddress (set-up, below) and only that address is used.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

alignas(256) uint8_t g_host_mask[kHostMaskBytes];
alignas(256) uint8_t g_host_stage[kHostStageBytes];

struct DeviceScratch {
    bool ready = false;
    unsigned char* ptr = nullptr;  // this device's copy of `scratch`
    hipEvent_t done = nullptr;     // recorded after each call's launch
    bool pending = false;          // `done` has been recorded
    Arena arena;
    Workspace ws;
};

// One call at a time in the process: the calls share the host staging, and
// the calls on one device share its scratch.
std::mutex g_mu;
DeviceScratch g_dev[kMaxDevices];

// Set-up on the current device, once: the address of its copy of the scratch
// and the event that orders a call after the previous one.
fse_status_t setup(int dev, DeviceScratch*& out) {
    if (dev < 0 || dev >= kMaxDevices) return FSE_ERR_UNSUPPORTED;
    DeviceScratch& D = g_dev[dev];
    if (!D.ready) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return FSE_ERR_DEVICE;
        e = hipEventCreateWithFlags(&D.done, hipEventDisableTiming);
        if (e != hipSuccess) return from_hip(e);
        D.ptr = (unsigned char*)p;
        D.arena.dev = D.ptr;
        D.arena.dev_cap = kScratchBytes;
        D.arena.host_mask = g_host_mask;
        D.arena.host_mask_cap = kHostMaskBytes;
        D.arena.host_stage = g_host_stage;
        D.arena.host_stage_cap = kHostStageBytes;
        D.ws.arena = &D.arena;
        D.ready = true;
    }
    out = &D;
    return FSE_OK;
}

}  // namespace

fse_status_t run_noalloc(const fse_image_t* image, const fse_mask_t* mask, const fse_params_t* p, fse_image_t* out,
                         hipStream_t st) {
    if (!image || !mask || !out) return FSE_ERR_INVALID_ARG;
    std::vector<ClassCfg> cls;
    if (!p) return FSE_ERR_INVALID_ARG;
    fse_status_t s = check_params(p, cls);
    if (s != FSE_OK) return s;
    // the FP64 working copy alone needs 8 bytes per pixel of every region
    if ((uint64_t)image->width * (uint64_t)image->height * 8 > kScratchBytes) return FSE_ERR_BUDGET;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return from_hip(e);
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceScratch* D = nullptr;
    if ((s = setup(dev, D)) != FSE_OK) return s;
    // the previous call on this device may still run on its own stream: its
    // kernels finish before this call overwrites the scratch
    if (D->pending && (e = hipEventSynchronize(D->done)) != hipSuccess) return from_hip(e);
    D->pending = false;
    std::lock_guard<std::mutex> wl(D->ws.mu);
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return from_hip(e);
    Prepared P;
    if ((s = prepare_batch(D->ws, 1, image, mask, p, out, cls, st, P)) != FSE_OK) return s;
    if ((s = launch_prepared(D->ws, P, st, false)) != FSE_OK) return s;
    if ((e = hipEventRecord(D->done, st)) != hipSuccess) return from_hip(e);
    D->pending = true;
    D->ws.last_stream = st;
    set_last_call_noalloc(P.stats, dev, st, D->done, (const int32_t*)D->ws.misc.p);
    return FSE_OK;
}

}  // namespace fse

extern "C" fse_status_t fse_extrapolate_noalloc(const fse_image_t* image, const fse_mask_t* mask,
                                                const fse_params_t* p, fse_image_t* out, void* stream) {
    return fse::abi_guard([&]() -> fse_status_t {
        return fse::run_noalloc(image, mask, p, out, (hipStream_t)stream);
    });
}
