// fse_internal.h -- structures shared by the host runtime and the gfx950
// kernels of libfse (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fse {

// One processing block per workgroup of 1, 2 or 4 wave64 (32 x 32 windows);
// launches that hold 64 x 64 windows use kWideWaves waves per workgroup.
constexpr int kWideWaves = 8;
constexpr int kMaxClasses = 3;

struct ClassDev {
    int32_t B, b, M, K;
    const double* wtab;  // M*M: rho^dist from the window centre (FP64)
};

// One job = one independently extrapolated region: a whole image, or one
// extended tile of the overlapping-tile framework.
struct JobDev {
    const float* img;     // source image (full-image coordinates)
    const uint8_t* mask;  // source mask
    float* out;           // destination image (full-image coordinates)
    int64_t img_pitch, mask_pitch, out_pitch;
    double* recon;    // region W*H: FP64 reconstructed values (valid where written)
    int32_t W, H;     // region size
    int32_t ox, oy;   // region origin in the source image
    int32_t cx0, cy0, cx1, cy1;  // core rectangle (region coords); output written only inside
    int32_t fw, fh;              // fine-cell grid of the region
    const int32_t* owner;        // fw*fh: block index owning the cell's lost pixels, -1 none
    const int4* desc;            // per block: y0, x0, class, 0 (region coords)
    const int4* lbox;            // per block: bounding box of its lost pixels [ly0,ly1) x [lx0,lx1)
    int32_t* done;               // per block completion flag
    int32_t n_blocks;
    int32_t trace_stride;
    int32_t* trace;              // may be null
    int64_t trace_cap;
};

struct LaunchArgs {
    const JobDev* jobs;
    const int2* tickets;  // (job, block) in dispatch order (a topological order)
    int32_t n_tickets;
    int32_t* counter;     // ticket dispenser, zero before launch
    int32_t* error;       // set non-zero when a dependency wait times out
    int64_t* degenerate;  // count of blocks with W0 == 0
    ClassDev cls[kMaxClasses];
    int32_t n_classes;
    int32_t Bmin;
    int32_t reach;        // max border over classes (px): edge test reach
    double gamma, delta;
    const double* tw32;   // cos, sin of 2 pi p / 32, p = 0..31 (64 doubles)
    const double* tw64;   // cos, sin of 2 pi p / 64 (128 doubles)
    int64_t wait_limit;   // dependency wait limit in s_memrealtime ticks (100 MHz)
};

// Launchers implemented in fse_kernels.hip.
hipError_t launch_init_job(const JobDev* jobs_dev, int n_jobs, int max_w, int max_h, int32_t* counter,
                           int32_t* error, int64_t* degenerate, hipStream_t st);
// grid workgroups; with a.counter set they draw tickets from the counter,
// otherwise workgroup g runs ticket ticket_base + g
hipError_t launch_blocks_at(const LaunchArgs& a, int nw, int prec, bool wide, int grid, int ticket_base,
                            hipStream_t st);
size_t shared_bytes_blocks(bool wide);

}  // namespace fse
