// fse_kernels.hip -- gfx950 kernels of Frequency Selective Extrapolation.
//
// One processing block per workgroup of one, two or four wave64 (eight in
// launches with 64 x 64 windows).  Per block:
//   1. stage the M x M support window from the mask, the plan and the image:
//      weights w = rho^dist (known pixels), delta rho^dist (pixels owned by an
//      earlier block, reconstructed by the time this one runs in raster
//      order), 0 (lost or outside); W0 = sum w; the known part of w*s; and
//      the DFT of w -- all of it fixed before any earlier block finishes;
//   2. wait until every earlier block that shares pixels with this block's
//      support window (in either direction) has finished, so the window holds
//      exactly what a strict raster-order pass would see;
//   3. add the reconstructed values to w*s and take its DFT; both DFTs are
//      F X F on the FP64 matrix cores (v_mfma_f64_16x16x4f64),
//      F[k,m] = e^{-2 pi i k m / M};
//   4. K greedy steps: argmax of |R|^2 (ties to the smallest index),
//      alpha = gamma R[u,v] / W0, R -= alpha * W shifted by (u,v) -- with
//      the weight spectrum stored pre-scaled by gamma / W0, so a step
//      subtracts R[u,v] times the stored spectrum and records R[u,v];
//   5. evaluate Re sum alpha e^{+2 pi i (u m + v n)/M} at the block's lost
//      pixels (gamma / W0 times the sum over the recorded R[u,v]), store
//      them (FP64 working copy and float32 output), publish.
// The block model is Sec. II of the paper; the wait and the persistent
// ticket dispatch are this library's way of running it on the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "fse_internal.h"
#include "fse_runtime.h"

namespace fse {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// working-state initialisation
// ---------------------------------------------------------------------------
// grid: x over columns, y over rows (strided), z over the jobs job0 ..
__global__ void k_init_job(const JobDev* __restrict__ jobs, int job0, int32_t* counter, int32_t* error,
                           int64_t* degenerate) {
    const JobDev& J = jobs[job0 + blockIdx.z];
    // clear the completion flags of this job's blocks
    const int64_t flat = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nflat = (int64_t)gridDim.x * gridDim.y * blockDim.x;
    for (int64_t i = flat; i < J.n_blocks; i += nflat) J.done[i] = 0;
    if (flat == 0 && job0 + blockIdx.z == 0) {
        if (counter) *counter = 0;
        *error = 0;
        *degenerate = 0;
    }
    for (int y = blockIdx.y; y < J.H; y += gridDim.y) {
        for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < J.W; x += gridDim.x * blockDim.x) {
            const int gy = J.oy + y, gx = J.ox + x;
            const uint8_t lost = J.mask[(int64_t)gy * J.mask_pitch + gx] != 0;
            if (!lost && y >= J.cy0 && y < J.cy1 && x >= J.cx0 && x < J.cx1)
                J.out[(int64_t)gy * J.out_pitch + gx] = J.img[(int64_t)gy * J.img_pitch + gx];
        }
    }
}

// One launch per 65535 jobs (the grid's z limit); rows strided over at most
// 4096 grid rows.  The launch holding job 0 also clears the shared counters.
hipError_t launch_init_job(const JobDev* jobs_dev, int n_jobs, int max_w, int max_h, int32_t* counter,
                           int32_t* error, int64_t* degenerate, hipStream_t st) {
    if (n_jobs <= 0) return hipSuccess;
    constexpr int kMaxZ = 65535, kMaxY = 4096;
    for (int job0 = 0; job0 < n_jobs; job0 += kMaxZ) {
        const int nz = std::min(kMaxZ, n_jobs - job0);
        dim3 grid((max_w + 255) / 256, std::min(max_h, kMaxY), nz);
        hipLaunchKernelGGL(k_init_job, grid, dim3(256), 0, st, jobs_dev, job0, counter, error, degenerate);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
// Loads of data that no kernel of the launch writes (job descriptors, block
// descriptors).  Through the constant address space a uniform address becomes
// a scalar load kept in SGPRs instead of repeated vector loads.
template <class T>
__device__ __forceinline__ T const_load(const T* p) {
#if defined(__HIP_DEVICE_COMPILE__)
    return *(const __attribute__((address_space(4))) T*)(p);
#else
    return *p;  // host pass: never executed, address spaces do not exist there
#endif
}

// Uniform loads of block-constant records (the job and block descriptors):
// each dword passes through readfirstlane, so the record lives in SGPRs for
// the whole block instead of occupying a VGPR per dword.  (The compiler
// otherwise turns these loads into per-lane vector loads.)
template <class T>
__device__ __forceinline__ T uniform_load(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "dword records");
    T r;
    const int32_t* s = reinterpret_cast<const int32_t*>(p);
    int32_t* d = reinterpret_cast<int32_t*>(&r);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) d[i] = __builtin_amdgcn_readfirstlane(const_load(s + i));
    return r;
}

// Completion flags are polled with relaxed loads; one acquire fence follows
// the wait.  (An acquire load per poll would invalidate caches on every
// iteration of the wait.)
__device__ __forceinline__ int ld_flag(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// s_waitcnt vmcnt(0): wait until this wave's vector memory operations have
// completed (expcnt and lgkmcnt left alone)
constexpr int kWaitVmcnt0 = 0x0F70;



__device__ __forceinline__ bool boxes_meet(int ay0, int ax0, int ay1, int ax1, int by0, int bx0, int by1,
                                           int bx1) {
    return ay0 < by1 && by0 < ay1 && ax0 < bx1 && bx0 < ax1;
}

// LDS layout.  M = 32: the area holds w*s (M x (M+1)), kept from before the
// dependency wait until the DFT of w*s after it, followed by a region that
// first holds w (M x (M+1)) and then the weight spectrum for the K steps
// ((32 + kWrapRows) x 32 complex, rows 0 .. kWrapRows-1 repeated after row
// 31); the coefficient list of the K steps takes the part of the area that
// the steps no longer read (32 KB with the head).  M = 64: w*s and w in two
// areas of 64 x 65; the weight spectrum (64 x 64 complex) stays in registers
// from its DFT (before the wait) until the DFT of w*s has read both areas,
// and is then written over them; the coefficient list follows (73 KB with
// the head, so that two blocks share a CU).
constexpr int kMaxK = 256;
// A lane's four elements of one row tile lie on rows base + ROWR r (r < 4,
// ROWR <= 4 rows): with the base reduced mod 32 they stay below 32 + 12.
constexpr int kWrapRows = 12;
constexpr int kBufDoubles32 = 32 * 33 + (32 + kWrapRows) * 32 * 2;  // w*s, then the weight spectrum
// M = 64: w*s and w in two areas of 64 x 65, the weight spectrum written over
// both once the DFT of w*s has read them, then the coefficient list
constexpr int kBufDoubles64 = 2 * 64 * 65 + 2 * kMaxK + kMaxK / 2;

struct SharedHead {
    double twc32[32], tws32[32];
    double part[8];
    // per step (three in rotation): the maximum over the waves of the wave
    // winner's energy with its last 12 bits replaced by 4095 - its index
    unsigned long long kmax[3];
    // per step (double-buffered) and wave: the wave winner's value R[u,v]
    double2 sA[2][8];
    int job, blk;
    uint8_t lost[16 * 16];  // lost pixels of the block's B x B core (B <= 16)
};

// 32 x 32 launches: the head and the buffer (32 KB in all, so the LDS of a CU
// holds five blocks, as does the 96-VGPR bound of the 4-wave kernels).
// Launches with 64 x 64 windows add the 64-point twiddles.
struct Shared32 {
    SharedHead h;
    double buf[kBufDoubles32];
};
struct Shared64 {
    SharedHead h;
    double tw64[128];  // cos, then sin, of 2 pi p / 64
    double buf[kBufDoubles64];
};
static_assert(sizeof(Shared32) <= 32768, "five 32 x 32 blocks per CU");
static_assert(2 * sizeof(Shared64) <= 160 * 1024, "two blocks of launches with 64 x 64 windows per CU");

// Unsigned 32-bit maximum over a wave64 with DPP; the result is valid in
// lane 63.  Non-negative doubles order like their bit patterns, so the high
// words of the energies order them up to ties in the high word.
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ unsigned dpp_umax_step(unsigned v) {
    // lanes without a source (and rows outside ROW_MASK) read 0, the identity
    const unsigned o = (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, BANK_MASK, false);
    return __builtin_elementwise_max(v, o);
}

__device__ __forceinline__ unsigned wave_umax(unsigned v) {
    v = dpp_umax_step<0xB1, 0xF, 0xF>(v);   // quad_perm [1,0,3,2]
    v = dpp_umax_step<0x4E, 0xF, 0xF>(v);   // quad_perm [2,3,0,1]
    v = dpp_umax_step<0x141, 0xF, 0xF>(v);  // row_half_mirror
    v = dpp_umax_step<0x140, 0xF, 0xF>(v);  // row_mirror
    v = dpp_umax_step<0x142, 0xA, 0xF>(v);  // row_bcast:15 into rows 1, 3
    v = dpp_umax_step<0x143, 0xC, 0xF>(v);  // row_bcast:31 into rows 2, 3
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// More than one lane in a (uniform) ballot: its population count in one
// scalar instruction (the compiler's form, a 64-bit x & (x - 1), takes four
// on the step's critical path)
__device__ __forceinline__ bool several_lanes(uint64_t bal) {
    int c;
    asm("s_bcnt1_i32_b64 %0, %1" : "=s"(c) : "s"(bal) : "scc");
    return c > 1;
}

// Lane holding the wave's largest non-negative energy; among equal energies
// the lane whose spectrum index is smallest.  The high words decide in one
// DPP pass unless several lanes share the largest high word.
template <class IndexFn>
__device__ __forceinline__ int wave_argmax_lane(double e, IndexFn idx_of) {
    const unsigned hi = (unsigned)__double2hiint(e);
    const unsigned mhi = wave_umax(hi);
    bool cand = hi == mhi;
    uint64_t bal = __ballot(cand);
    if (several_lanes(bal)) {
        const unsigned lo = (unsigned)__double2loint(e);
        const unsigned mlo = wave_umax(cand ? lo : 0u);
        cand = cand && lo == mlo;
        bal = __ballot(cand);
        if (several_lanes(bal)) {
            // exact tie between lanes: the smallest spectrum index among them,
            // as the DPP maximum of its complement (no shuffle addresses to
            // keep in registers)
            const unsigned inv = cand ? ~(unsigned)idx_of() : 0u;
            const unsigned minv = wave_umax(inv);  // with every lane active
            bal = __ballot(cand && inv == minv);
        }
    }
    // bal is never empty (some lane holds the maximum): the first set bit
    // without a zero test
    return __builtin_amdgcn_readfirstlane(__builtin_ctzll((unsigned long long)bal));
}

template <class IndexFn>
__device__ __forceinline__ int wave_argmax_lane(float e, IndexFn idx_of) {
    const unsigned k = __float_as_uint(e);
    const bool cand = k == wave_umax(k);
    uint64_t bal = __ballot(cand);
    if (several_lanes(bal)) {
        const unsigned inv = cand ? ~(unsigned)idx_of() : 0u;
        const unsigned minv = wave_umax(inv);  // with every lane active
        bal = __ballot(cand && inv == minv);
    }
    // bal is never empty (some lane holds the maximum): the first set bit
    // without a zero test
    return __builtin_amdgcn_readfirstlane(__builtin_ctzll((unsigned long long)bal));
}

__device__ __forceinline__ double readlane_t(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ __forceinline__ float readlane_t(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}



// ---------------------------------------------------------------------------
// precision policies
//   kPrecF64    : FP64 MFMA DFT, FP64 selection loop (the parity path)
//   kPrecF32    : FP32 MFMA DFT, FP32 loop
//   kPrecBF16x3 : DFT with BF16 hi/lo splits of both operands, three BF16
//                 MFMAs per product (hi*hi + hi*lo + lo*hi), FP32 accumulate;
//                 FP32 loop
// W0, the coefficients alpha, the synthesis and the reconstructed values stay
// FP64 in every policy.
// ---------------------------------------------------------------------------
constexpr int kPrecF64 = 0, kPrecF32 = 1, kPrecBF16x3 = 2;
template <int PREC> struct PrecType { using T = float; };
template <> struct PrecType<kPrecF64> { using T = double; };

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef short bf4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ short bf16_bits(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}
__device__ __forceinline__ float bf16_value(short h) { return __uint_as_float(((unsigned)(unsigned short)h) << 16); }
// x ~ hi + lo with both in bfloat16
__device__ __forceinline__ void bf16_split(float x, short& hi, short& lo) {
    hi = bf16_bits(x);
    lo = bf16_bits(x - bf16_value(hi));
}

// one accumulating product step of the DFT for each policy; a and b are the
// operands of this lane (the BF16 policy passes four consecutive k values)
__device__ __forceinline__ dbl4 mfma_step(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ flt4 mfma_step(float a, float b, flt4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ flt4 mfma_step3(const float (&a)[4], const float (&b)[4], flt4 c) {
    bf4 ah, al, bh, bl;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        short h, l;
        bf16_split(a[q], h, l);
        ah[q] = h;
        al[q] = l;
        bf16_split(b[q], h, l);
        bh[q] = h;
        bl[q] = l;
    }
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, c, 0, 0, 0);
    return c;
}

// ---------------------------------------------------------------------------
// one block with an M x M window (M = 32 or 64), NW wave64 per block,
// arithmetic policy PREC
//
// DFT dataflow: stage 1 forms T = X F (A operand X from LDS, B operand the
// twiddles), stage 2 forms F T with the B operand taken straight from the
// stage-1 accumulators, which already hold T in the lane layout of the B
// operand once the contraction index of stage 2 is ordered to match (FP64
// output rows are lane/16 + 4r; FP32 and BF16 output rows are 4(lane/16) + r).
// Each wave owns NTI x NTJ output tiles of 16 x 16; it computes the stage-1
// columns it needs for both inputs (w*s and w), keeps its tiles of R in
// registers for the K steps and writes its tiles of the weight spectrum to
// LDS.
// ---------------------------------------------------------------------------
template <int M, int NW>
struct TileMap {
    static constexpr int TL = M / 16;  // tiles per dimension
    // column tiles per wave
    static constexpr int NTJ = (M == 32) ? ((NW == 1) ? 2 : 1) : ((NW <= 4) ? 4 / NW : 1);
    // row tiles per wave
    static constexpr int NTI = (M == 32) ? ((NW == 4) ? 1 : 2) : ((NW <= 4) ? 4 : 2);
    __host__ __device__ static constexpr int ti0(int wv) {
        return (M == 32) ? ((NW == 4) ? (wv >> 1) : 0) : ((NW == 8) ? (wv >> 2) * 2 : 0);
    }
    __host__ __device__ static constexpr int tj0(int wv) {
        return (M == 32) ? ((NW == 4) ? (wv & 1) : (NW == 2 ? wv : 0)) : ((NW == 8) ? (wv & 3) : wv * NTJ);
    }
    // the wave that owns spectrum tile (row tile rt, column tile ct)
    __host__ __device__ static constexpr int wave_of(int rt, int ct) {
        return (M == 32) ? ((NW == 4) ? ((rt << 1) | ct) : (NW == 2 ? ct : 0))
                         : ((NW == 8) ? (((rt >> 1) << 2) | ct) : ct / NTJ);
    }
    static constexpr bool wave_of_inverts() {
        for (int w = 0; w < NW; ++w)
            for (int i = 0; i < NTI; ++i)
                for (int j = 0; j < NTJ; ++j)
                    if (wave_of(ti0(w) + i, tj0(w) + j) != w) return false;
        return true;
    }
};

template <int NT>
__device__ void wait_predecessors(const LaunchArgs& a, const JobDev& J, int blk);

// NW waves compute the DFT and the K steps; the workgroup has NWG >= NW
// waves, all of which stage the window, wait and synthesise (waves past NW
// only keep the barriers of the DFT and the K steps).
template <int M, int NW, int NWG, int PREC>
__device__ void process_block(const LaunchArgs& a, const JobDev& J, int blk, SharedHead& H, double* buf,
                              const double* tw64) {
    using T = typename PrecType<PREC>::T;
    using acc4 = typename std::conditional<PREC == kPrecF64, dbl4, flt4>::type;
    using TM = TileMap<M, NW>;
    constexpr bool F64 = PREC == kPrecF64;
    constexpr int NT = 64 * NWG;              // threads
    constexpr int NTJ = TM::NTJ, NTI = TM::NTI;
    constexpr int EPT = NTI * NTJ * 4;        // spectrum elements per lane
    constexpr int NPIX = M * M / NT;          // window pixels per thread while staging
    constexpr int RS = NT / M;                // window-row step between a thread's pixels
    constexpr int KK = M / 4;                 // k-steps of a 16x16x4 product
    constexpr int KB = M / 16;                // k-steps of a 16x16x16 product
    constexpr int LD = M + 1;                 // padded row stride of X
    constexpr int MASK = M - 1;
    constexpr int LOGM = (M == 32) ? 5 : 6;
    constexpr bool DUP = (M == 32);           // weight spectrum rows 0 .. kWrapRows-1 repeated after row M-1
    const double* twc = (M == 32) ? H.twc32 : tw64;
    const double* tws = (M == 32) ? H.tws32 : tw64 + 64;
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);  // in a scalar register
    const bool active = wv < NW;  // wave-uniform
    const int ti0 = TM::ti0(wv), tj0 = TM::tj0(wv);
    const int4 d = uniform_load(J.desc + blk);
    const ClassDev& C = a.cls[d.z];
    const int B = C.B, b = C.b, K = C.K;
    const int wy = d.x - b, wx = d.y - b;  // window origin (region coords); desc = (y0, x0, cls, 0)

    __builtin_amdgcn_s_setprio(0);  // staging before the wait: lowest issue priority
    // ---- stage the window: weights and weighted values --------------------
    // A window pixel is known (weight rho^dist), lost and owned by an earlier
    // block (reconstructed by the time this block runs in raster order:
    // delta rho^dist), or lost otherwise (0) -- fixed by the mask and the plan,
    // so the weights, W0, the known part of w*s and the weight spectrum are
    // formed before the dependency wait; only the reconstructed values wait.
    // M = 64 keeps the weight spectrum in registers until both staged areas
    // have been read (see the LDS layout above)
    constexpr bool WREG = (M == 64);
    T* Xs = reinterpret_cast<T*>(buf);           // w * s, [m][n] stride LD
    T* Wd = WREG ? Xs : Xs + M * LD;             // weight spectrum [DUP ? M + kWrapRows : M][M] complex
    T* Xw = WREG ? Xs + M * LD : Wd;             // w (M = 32: staged where the weight spectrum goes)
    // coefficient list of the K steps (real parts, imaginary parts, spectrum
    // indices; the values are R[u,v], each coefficient is gamma / W0 times
    // its value), written during the steps and read by the synthesis: M = 32
    // in FP64 over w*s, which the steps no longer read, in FP32 after the
    // weight spectrum, where the buffer (sized for FP64) is free; M = 64
    // after the two staged areas
    constexpr int kWdRows = DUP ? M + kWrapRows : M;
    static_assert(WREG ? (2 * M * LD + 2 * kMaxK + kMaxK / 2 <= kBufDoubles64 && M * M * 2 * sizeof(T) <= 2 * M * LD * sizeof(double))
                       : F64 ? 2 * kMaxK + kMaxK / 2 <= M * LD
                             : (M * LD + kWdRows * M * 2) / 2 + 2 * kMaxK + kMaxK / 2 <= kBufDoubles32,
                  "coefficient list inside the buffer");
    double* const clist = WREG ? buf + 2 * M * LD : F64 ? buf : reinterpret_cast<double*>(Wd + kWdRows * M * 2);
    double* const car = clist;
    double* const cai = clist + kMaxK;
    int32_t* const cidx = reinterpret_cast<int32_t*>(clist + 2 * kMaxK);
    const int Bm = a.Bmin;
    double wsum = 0.0;
    unsigned recon_bits = 0;  // this thread's pixels that hold reconstructed values
#pragma unroll
    for (int j = 0; j < NPIX; ++j) {
        const int m = (t >> LOGM) + RS * j, n = t & MASK;
        const int y = wy + m, x = wx + n;
        double w = 0.0, v = 0.0;
        bool lost = false;
        if (y >= 0 && y < J.H && x >= 0 && x < J.W) {
            // independent loads, in flight together
            lost = J.mask[(int64_t)(J.oy + y) * J.mask_pitch + (J.ox + x)] != 0;
            const int own = J.owner[(y / Bm) * J.fw + x / Bm];
            const double wt = C.wtab[m * M + n];
            const double sv = (double)J.img[(int64_t)(J.oy + y) * J.img_pitch + (J.ox + x)];
            const bool rec = lost && own < blk;
            w = !lost ? wt : (rec ? a.delta * wt : 0.0);
            v = !lost ? sv : 0.0;
            recon_bits |= (unsigned)rec << j;
        }
        Xs[m * LD + n] = (T)(w * v);
        Xw[m * LD + n] = (T)w;
        wsum += w;
        // lost pixels of the core, synthesised at the end
        if (m >= b && m < b + B && n >= b && n < b + B) H.lost[(m - b) * B + (n - b)] = lost;
    }
    for (int off = 32; off >= 1; off >>= 1) wsum += __shfl_xor(wsum, off);
    if (lane == 0) H.part[wv] = wsum;
    __syncthreads();  // the per-wave sums of w stay in LDS until the steps need W0
    // gamma / W0 from the per-wave sums (0 for a block without known
    // pixels), formed where it is needed rather than held in registers
    auto gain = [&]() {
        double W0 = H.part[0];
#pragma unroll
        for (int q = 1; q < NWG; ++q) W0 += H.part[q];
        return W0 > 0.0 ? a.gamma / W0 : 0.0;
    };

    // ---- DFT of one input (1: w -> weight spectrum in LDS, 0: w*s -> R in
    // registers) as F X F in two stages of MFMA GEMMs
    // stage 1: T(:, tj) = X F(:, tj); F = C - i S with C[k,m] = cos(2 pi k m / M),
    // S[k,m] = sin(2 pi k m / M)
    const int li = lane & 15, lk = lane >> 4;
    T rr[EPT], ri[EPT];
    auto dft = [&](const int inp) {
    // the lane coordinates again, opaque to the compiler: the per-lane twiddle
    // addresses derived from them are recomputed in each DFT (a few integer
    // operations) instead of being hoisted out of the block loop, where they
    // would hold two dozen registers for the whole loop
    int li = lane & 15, lk = lane >> 4;
    asm volatile("" : "+v"(li), "+v"(lk));
    acc4 t1[NTJ][TM::TL][2];  // [column tile][row tile][re, im]
    if (active) {
        const T* X = inp ? Xw : Xs;
#pragma unroll
        for (int cj = 0; cj < NTJ; ++cj) {
            const int tj = tj0 + cj;
#pragma unroll
            for (int ti = 0; ti < TM::TL; ++ti) {
                acc4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
                if constexpr (PREC == kPrecBF16x3) {
#pragma unroll
                    for (int kk = 0; kk < KB; ++kk) {
                        float av[4], bc[4], bs[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int k = kk * 16 + 4 * lk + q;
                            av[q] = X[(ti * 16 + li) * LD + k];
                            const int p = (k * (tj * 16 + li)) & MASK;
                            bc[q] = (float)twc[p];
                            bs[q] = -(float)tws[p];
                        }
                        cr = mfma_step3(av, bc, cr);
                        ci = mfma_step3(av, bs, ci);
                    }
                } else {
#pragma unroll
                    for (int kk = 0; kk < KK; ++kk) {
                        const T av = X[(ti * 16 + li) * LD + kk * 4 + lk];
                        const int p = ((kk * 4 + lk) * (tj * 16 + li)) & MASK;
                        cr = mfma_step(av, (T)twc[p], cr);
                        ci = mfma_step(av, (T)(-tws[p]), ci);
                    }
                }
                t1[cj][ti][0] = cr;
                t1[cj][ti][1] = ci;
            }
        }
    }
    if (inp == 1) __syncthreads();  // w is dead; the weight spectrum takes its place

    // stage 2: F T for the wave's tiles; (F T)_re = C T_re + S T_im,
    // (F T)_im = C T_im - S T_re
    const double g1 = inp == 1 ? gain() : 0.0;
    if (active) {
#pragma unroll
        for (int ci_ = 0; ci_ < NTI; ++ci_) {
#pragma unroll
            for (int cj = 0; cj < NTJ; ++cj) {
                const int ti_o = ti0 + ci_, tj = tj0 + cj;
                acc4 ore = {0, 0, 0, 0}, oim = {0, 0, 0, 0};
                if constexpr (PREC == kPrecBF16x3) {
#pragma unroll
                    for (int kk = 0; kk < KB; ++kk) {
                        float c[4], sn[4], nsn[4], bre[4], bim[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int k = kk * 16 + 4 * lk + q;
                            const int p = ((ti_o * 16 + li) * k) & MASK;
                            c[q] = (float)twc[p];
                            sn[q] = (float)tws[p];
                            nsn[q] = -sn[q];
                            bre[q] = t1[cj][kk][0][q];
                            bim[q] = t1[cj][kk][1][q];
                        }
                        ore = mfma_step3(c, bre, ore);
                        ore = mfma_step3(sn, bim, ore);
                        oim = mfma_step3(c, bim, oim);
                        oim = mfma_step3(nsn, bre, oim);
                    }
                } else {
#pragma unroll
                    for (int kk = 0; kk < KK; ++kk) {
                        // contraction index held by this lane in accumulator kk
                        const int k = F64 ? (kk * 4 + lk) : ((kk >> 2) * 16 + 4 * lk + (kk & 3));
                        const int p = ((ti_o * 16 + li) * k) & MASK;
                        const T c = (T)twc[p], sn = (T)tws[p];
                        const T bre = t1[cj][kk >> 2][0][kk & 3];
                        const T bim = t1[cj][kk >> 2][1][kk & 3];
                        ore = mfma_step(c, bre, ore);
                        ore = mfma_step(sn, bim, ore);
                        oim = mfma_step(c, bim, oim);
                        oim = mfma_step((T)(-sn), bre, oim);
                    }
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int k = ti_o * 16 + (F64 ? (lk + 4 * r) : (4 * lk + r)), l = tj * 16 + li;
                    if (inp == 1) {
                        // the weight spectrum scaled by gamma / W0
                        const T sre = (T)(g1 * (double)ore[r]), sim = (T)(g1 * (double)oim[r]);
                        Wd[(k * M + l) * 2] = sre;
                        Wd[(k * M + l) * 2 + 1] = sim;
                        if (DUP && k < kWrapRows) {
                            Wd[((k + M) * M + l) * 2] = sre;
                            Wd[((k + M) * M + l) * 2 + 1] = sim;
                        }
                    } else {
                        // element order within a lane = increasing spectrum index
                        const int e = (ci_ * 4 + r) * NTJ + cj;
                        rr[e] = ore[r];
                        ri[e] = oim[r];
                    }
                }
            }
        }
    }
    };

    // M = 64: the DFT streams over the row tiles kt of the first-stage product
    // T = X F -- each tile (kt, tj) is formed and at once contracted into
    // the wave's output tiles (its share of the second stage's sum runs over
    // k in tile kt) -- so only one tile of T is held at a time; the outputs
    // go to registers: the weight spectrum (held until both staged areas
    // have been read) or R
    T wrr[WREG ? EPT : 1], wri[WREG ? EPT : 1];
    auto dft_stream = [&](const int inp) {
        int li = lane & 15, lk = lane >> 4;
        asm volatile("" : "+v"(li), "+v"(lk));
        acc4 o_re[NTI][NTJ], o_im[NTI][NTJ];
#pragma unroll
        for (int ci_ = 0; ci_ < NTI; ++ci_)
#pragma unroll
            for (int cj = 0; cj < NTJ; ++cj) {
                o_re[ci_][cj] = acc4{0, 0, 0, 0};
                o_im[ci_][cj] = acc4{0, 0, 0, 0};
            }
        if (!active) return;
        const T* X = inp ? Xw : Xs;
#pragma unroll
        for (int kt = 0; kt < TM::TL; ++kt) {
            // opaque per tile: the twiddles (the same for every kt) are read
            // again for each tile instead of being held across all four
            asm volatile("" : "+v"(li), "+v"(lk));
#pragma unroll
            for (int cj = 0; cj < NTJ; ++cj) {
                const int tj = tj0 + cj;
                acc4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
                if constexpr (PREC == kPrecBF16x3) {
#pragma unroll
                    for (int kk = 0; kk < KB; ++kk) {
                        float av[4], bc[4], bs[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int k = kk * 16 + 4 * lk + q;
                            av[q] = X[(kt * 16 + li) * LD + k];
                            const int p = (k * (tj * 16 + li)) & MASK;
                            bc[q] = (float)twc[p];
                            bs[q] = -(float)tws[p];
                        }
                        cr = mfma_step3(av, bc, cr);
                        ci = mfma_step3(av, bs, ci);
                    }
#pragma unroll
                    for (int ci_ = 0; ci_ < NTI; ++ci_) {
                        const int ti_o = ti0 + ci_;
                        float c[4], sn[4], nsn[4], bre[4], bim[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int k = kt * 16 + 4 * lk + q;
                            const int p = ((ti_o * 16 + li) * k) & MASK;
                            c[q] = (float)twc[p];
                            sn[q] = (float)tws[p];
                            nsn[q] = -sn[q];
                            bre[q] = cr[q];
                            bim[q] = ci[q];
                        }
                        o_re[ci_][cj] = mfma_step3(c, bre, o_re[ci_][cj]);
                        o_re[ci_][cj] = mfma_step3(sn, bim, o_re[ci_][cj]);
                        o_im[ci_][cj] = mfma_step3(c, bim, o_im[ci_][cj]);
                        o_im[ci_][cj] = mfma_step3(nsn, bre, o_im[ci_][cj]);
                    }
                } else {
#pragma unroll
                    for (int kk = 0; kk < KK; ++kk) {
                        const T av = X[(kt * 16 + li) * LD + kk * 4 + lk];
                        const int p = ((kk * 4 + lk) * (tj * 16 + li)) & MASK;
                        cr = mfma_step(av, (T)twc[p], cr);
                        ci = mfma_step(av, (T)(-tws[p]), ci);
                    }
#pragma unroll
                    for (int ci_ = 0; ci_ < NTI; ++ci_) {
                        const int ti_o = ti0 + ci_;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            // contraction index held by this lane in accumulator q of tile kt
                            const int kk = kt * 4 + q;
                            const int k = F64 ? (kk * 4 + lk) : ((kk >> 2) * 16 + 4 * lk + (kk & 3));
                            const int p = ((ti_o * 16 + li) * k) & MASK;
                            const T c = (T)twc[p], sn = (T)tws[p];
                            o_re[ci_][cj] = mfma_step(c, cr[q], o_re[ci_][cj]);
                            o_re[ci_][cj] = mfma_step(sn, ci[q], o_re[ci_][cj]);
                            o_im[ci_][cj] = mfma_step(c, ci[q], o_im[ci_][cj]);
                            o_im[ci_][cj] = mfma_step((T)(-sn), cr[q], o_im[ci_][cj]);
                        }
                    }
                }
            }
        }
        // element order within a lane = increasing spectrum index
#pragma unroll
        for (int ci_ = 0; ci_ < NTI; ++ci_)
#pragma unroll
            for (int cj = 0; cj < NTJ; ++cj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int e = (ci_ * 4 + r) * NTJ + cj;
                    if (inp == 1) {
                        wrr[e] = o_re[ci_][cj][r];
                        wri[e] = o_im[ci_][cj][r];
                    } else {
                        rr[e] = o_re[ci_][cj][r];
                        ri[e] = o_im[ci_][cj][r];
                    }
                }
    };

    if constexpr (WREG)
        dft_stream(1);  // weight spectrum into registers, before the wait
    else
        dft(1);  // weight spectrum, before the wait

    // ---- wait for the earlier blocks this block depends on, then add their
    // reconstructed values to w*s
    wait_predecessors<NT>(a, J, blk);
    // from here on the block is ready work: its waves issue ahead of the
    // pre-wait staging of other blocks on the same SIMDs
    __builtin_amdgcn_s_setprio(3);
    // the pixel coordinates again, opaque to the compiler: the addresses are
    // recomputed here instead of being kept from the staging across the DFT
    int tp = t;
    asm volatile("" : "+v"(tp));
#pragma unroll
    for (int j = 0; j < NPIX; ++j) {
        if (recon_bits >> j & 1) {
            const int m = (tp >> LOGM) + RS * j, n = tp & MASK;
            const int64_t q = (int64_t)(wy + m) * J.W + (wx + n);
            Xs[m * LD + n] = (T)(a.delta * C.wtab[m * M + n] * J.recon[q]);
        }
    }
    __syncthreads();
    if constexpr (WREG) {
        dft_stream(0);  // R
        __syncthreads();  // both staged areas read: the weight spectrum takes them
        if (active) {
            const double g1 = gain();
            int li = lane & 15, lk = lane >> 4;
#pragma unroll
            for (int ci_ = 0; ci_ < NTI; ++ci_)
#pragma unroll
                for (int cj = 0; cj < NTJ; ++cj)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int e = (ci_ * 4 + r) * NTJ + cj;
                        const int k = (ti0 + ci_) * 16 + (F64 ? (lk + 4 * r) : (4 * lk + r)), l = (tj0 + cj) * 16 + li;
                        // the weight spectrum scaled by gamma / W0
                        Wd[(k * M + l) * 2] = (T)(g1 * (double)wrr[e]);
                        Wd[(k * M + l) * 2 + 1] = (T)(g1 * (double)wri[e]);
                    }
        }
    } else {
        dft(0);  // R
    }
    if (t == 0) H.kmax[0] = H.kmax[1] = H.kmax[2] = 0ull;  // the steps' maxima
    __syncthreads();

    // ---- K greedy steps ----------------------------------------------------
    // lane element e = (row tile ci_, r, column tile cj); its row is
    // (ti0+ci_)*16 + lk + 4r (FP64) or (ti0+ci_)*16 + 4 lk + r (FP32, BF16),
    // column (tj0+cj)*16 + li; the index k*M + l increases with e.
    // Per step: a first-index maximum inside the lane, the wave's winner lane
    // from a DPP maximum, the winner's values broadcast with readlane; with
    // several waves one LDS exchange (one barrier) combines the wave winners;
    // then the shifted weight spectrum is gathered from LDS for the update.
    constexpr int ROWK = F64 ? 1 : 4;  // row step per lk
    constexpr int ROWR = F64 ? 4 : 1;  // row step per r
    static_assert(!DUP || 3 * ROWR <= kWrapRows, "wrapped weight-spectrum rows");
    // W0 from the per-wave sums (read here rather than before the DFTs and
    // the wait, across which it would occupy registers)
    double W0 = H.part[0];
#pragma unroll
    for (int q = 1; q < NWG; ++q) W0 += H.part[q];
    // uniform across the block: lets the loop run under scalar control
    const bool live = __builtin_amdgcn_readfirstlane((int)(W0 > 0.0)) != 0;
    const int nsteps = live ? __builtin_amdgcn_readfirstlane(K) : 0;
    int32_t* trace = (J.trace && blk < J.trace_cap) ? J.trace + (int64_t)blk * J.trace_stride : nullptr;
    // the lane coordinates again, opaque to the compiler: the steps' per-lane
    // constants below are formed here, per block, instead of being kept in
    // registers across the DFTs (where they were spilled and reloaded)
    int sl = lane;
    asm volatile("" : "+v"(sl));
    const int sli = sl & 15, slk = sl >> 4;
    // spectrum index of lane element e = lane_idx + elem_offset(e)
    const int lane_idx = (ti0 * 16 + ROWK * slk) * M + tj0 * 16 + sli;
    // 4095 - lane_idx: the key's last 12 bits are 4095 - (lane_idx + elem_offset(e))
    const int lane_key = 0xFFF - lane_idx;
    auto elem_offset = [](int e) {
        const int jr = (e / NTJ) & 3, jci = e / (4 * NTJ), jcj = e % NTJ;
        return (jci * 16 + ROWR * jr) * M + jcj * 16;
    };
    // gather address of the shifted weight spectrum (M = 32, rows repeated,
    // one tile per wave): one base per lane for its four rows, (row mod M,
    // column mod M) formed as two 16-bit fields in one packed subtraction --
    // the row field in units of a spectrum row, the column field in units of
    // an element
    constexpr int ES = 2 * (int)sizeof(T);  // bytes per complex element
    constexpr bool PACKED = DUP && NTI == 1 && NTJ == 1;
    static_assert(!PACKED || (M - 1) * M * ES < 65536, "packed gather address");
    typedef unsigned short ushort2_v __attribute__((ext_vector_type(2)));
    const unsigned gather_base =
        ((unsigned)((ti0 * 16 + ROWK * slk) * M * ES) << 16) | (unsigned)((tj0 * 16 + sli) * ES);
    constexpr unsigned kGatherMask = ((unsigned)(MASK * M * ES) << 16) | (unsigned)(MASK * ES);
    // one selection step; P is the parity of the step (double-buffered
    // slots), Q the step mod 3 (the maximum it uses) when known at compile
    // time, else -1
    auto step = [&](const int it, auto parity, auto rot) {
        constexpr int P = decltype(parity)::value;
        constexpr int Q = decltype(rot)::value;
        // first-index maximum over the lane's elements (pairwise tree over
        // increasing index: the right operand wins only when strictly larger);
        // the tree carries the element's number (small constants, no
        // registers), with four elements per lane also its value; the
        // spectrum index follows from the number
        constexpr bool CARRY = EPT <= 4 || NW == 1;
        T ev[EPT], vr[CARRY ? EPT : 1], vi[CARRY ? EPT : 1];
        int ex[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            ev[j] = rr[j] * rr[j] + ri[j] * ri[j];
            if constexpr (CARRY) {
                vr[j] = rr[j];
                vi[j] = ri[j];
            }
            ex[j] = j;
        }
#pragma unroll
        for (int st = 1; st < EPT; st <<= 1) {
#pragma unroll
            for (int j = 0; j + st < EPT; j += 2 * st) {
                const bool take = ev[j + st] > ev[j];
                // the larger energy (equal ones are the same value): one
                // maximum instead of a select per word
                ev[j] = fmax(ev[j], ev[j + st]);
                ex[j] = take ? ex[j + st] : ex[j];
                if constexpr (CARRY) {
                    vr[j] = take ? vr[j + st] : vr[j];
                    vi[j] = take ? vi[j + st] : vi[j];
                }
            }
        }
        const T lm = ev[0];
        // 4095 - the spectrum index of the lane's maximum (the low bits of its
        // exchange key), and the index itself
        const int kx = lane_key - elem_offset(ex[0]);
        int ix[1] = {0xFFF - kx};
        double car_l, cai_l;
        if constexpr (CARRY) {
            // the lane's candidate value R (the step's coefficient is
            // gamma / W0 times it: that factor is in the stored weight
            // spectrum and in the synthesis), selected and in FP64 before
            // the wave reduction, so that it is ready when the winner lane
            // publishes it (the empty asm keeps the tree's value selects out
            // of the winner's branch)
            car_l = (double)vr[0];
            cai_l = (double)vi[0];
            asm volatile("" : "+v"(car_l), "+v"(cai_l));
        }
        // winner lane of the wave: largest energy, then smallest index
        const int wl = wave_argmax_lane(lm, [&] { return ix[0]; });
        if constexpr (!CARRY) {
            // more elements per lane: the winner's element number in a scalar
            // register selects its value by register index, instead of a
            // select per tree node and element
            const int ew = __builtin_amdgcn_readlane(ex[0], wl);
            car_l = (double)rr[ew];
            cai_l = (double)ri[ew];
        }
        int IDX;
        double ar, ai;
        if constexpr (NW == 1) {
            IDX = __builtin_amdgcn_readlane(ix[0], wl);
            ar = readlane_t(car_l, wl);
            ai = readlane_t(cai_l, wl);
        } else {
            // the block winner through one 64-bit LDS maximum: each wave's
            // winner lane enters its non-negative energy (whose bit pattern
            // orders like its value) with the last 12 bits replaced by
            // 4095 - its index, so equal energies, and energies within 2^-40
            // of each other, go to the smaller index; and it publishes its
            // value R[u,v].  Three maxima rotate: the one of the step after
            // this is cleared now (its last readers, two steps back, have all
            // passed the previous barrier, and no wave enters it before this
            // step's barrier).
            static_assert(TM::wave_of_inverts(), "tile owner");
            const int ks = Q >= 0 ? Q : it % 3, kn = Q >= 0 ? (Q + 1) % 3 : (it + 1) % 3;
            if (lane == wl) {
                const unsigned long long key =
                    ((unsigned long long)__double_as_longlong((double)lm) & ~0xFFFull) | (unsigned long long)(unsigned)kx;
                atomicMax(&H.kmax[ks], key);
                H.sA[P][wv] = make_double2(car_l, cai_l);
                // every wave's winner lane clears the same maximum (the
                // same value written NW times; no condition to evaluate)
                H.kmax[kn] = 0ull;
            }
            __syncthreads();  // the maximum and the coefficients visible to every wave
            const unsigned long long km = H.kmax[ks];
            IDX = 0xFFF - (__builtin_amdgcn_readfirstlane((int)(unsigned)km) & 0xFFF);
            const int wq = TM::wave_of((IDX >> LOGM) >> 4, (IDX & MASK) >> 4);
            const double2 al = H.sA[P][wq];
            ar = al.x;
            ai = al.y;
        }
        // the shifted weight spectrum for this lane's elements
        const int u = IDX >> LOGM, v = IDX & MASK;
        T wr[EPT], wi[EPT];
        if constexpr (PACKED) {
            const unsigned shift = ((unsigned)(u * M * ES) << 16) | (unsigned)(v * ES);
            const ushort2_v d = __builtin_bit_cast(ushort2_v, gather_base) - __builtin_bit_cast(ushort2_v, shift);
            const unsigned f = __builtin_bit_cast(unsigned, d) & kGatherMask;
            const unsigned char* w0 = reinterpret_cast<const unsigned char*>(Wd) + (f >> 16) + (f & 0xffffu);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                // rows (row0 mod M) + ROWR r lie below M + kWrapRows
                const T* w = reinterpret_cast<const T*>(w0 + r * (ROWR * M * ES));
                wr[r] = w[0];
                wi[r] = w[1];
            }
        } else {
#pragma unroll
            for (int ci_ = 0; ci_ < NTI; ++ci_) {
#pragma unroll
                for (int cj = 0; cj < NTJ; ++cj) {
                    const int col = ((tj0 + cj) * 16 + sli - v) & MASK;
                    const int row0 = (ti0 + ci_) * 16 + ROWK * slk - u;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int e = (ci_ * 4 + r) * NTJ + cj;
                        // DUP: rows (row0 mod M) + ROWR r lie below M + kWrapRows
                        const T* w = DUP ? (Wd + (((row0 & MASK) << LOGM) + col) * 2 + r * (ROWR * M * 2))
                                         : (Wd + ((((row0 + ROWR * r) & MASK) << LOGM) + col) * 2);
                        wr[e] = w[0];
                        wi[e] = w[1];
                    }
                }
            }
        }
        const T tar = (T)ar, tai = (T)ai;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            rr[e] = fma(-tar, wr[e], fma(tai, wi[e], rr[e]));
            ri[e] = fma(-tar, wi[e], fma(-tai, wr[e], ri[e]));
        }
        // the step's value and index, recorded off the critical path (read
        // only after the loop)
        if (t == 0) {
            car[it] = ar;
            cai[it] = ai;
            cidx[it] = IDX;
        }
    };
    if (!active) {
        if constexpr (NW > 1)
            for (int it = 0; it < nsteps; ++it) __syncthreads();  // the step exchanges of the active waves
    } else {
        // unrolled by six, so that the slot and maximum offsets are constants
        // (FP64; the FP32 loops stay unrolled by two: with nine copies of the
        // step the compiler kept them out of line, their arrays in scratch)
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        using IN = std::integral_constant<int, -1>;
        int it = 0;
        if constexpr (F64) {
            for (; it + 6 <= nsteps; it += 6) {
                step(it, I0(), I0());
                step(it + 1, I1(), I1());
                step(it + 2, I0(), I2());
                step(it + 3, I1(), I0());
                step(it + 4, I0(), I1());
                step(it + 5, I1(), I2());
            }
        }
        for (; it + 1 < nsteps; it += 2) {
            step(it, I0(), IN());
            step(it + 1, I1(), IN());
        }
        if (it < nsteps) step(it, I0(), IN());
    }
    if (!live && t == 0) atomicAdd((unsigned long long*)a.degenerate, 1ull);
    __syncthreads();  // the coefficient list is complete
    if (trace)
        for (int it = t; it < nsteps; it += NT) trace[it] = cidx[it];

    // ---- synthesis at the block's lost pixels ------------------------------
    const double g = gain();
    // gs lanes of one wave per pixel, each summing every gs-th step; B*B
    // pixels.  gs stays within a wave (at most 64): the lane sums are
    // combined with shuffles, which do not cross waves.
    const int npx = B * B;
    const int gs = npx >= NT ? 1 : min(64, NT / npx);
    const int sub = t % gs;
    for (int px = t / gs; px < npx; px += NT / gs) {
        const int py = px / B, pxx = px % B;
        const int m = b + py, n = b + pxx;
        double val = 0.0;
        if (live) {
            for (int it = sub; it < K; it += gs) {
                const int idx = cidx[it];
                const int u = idx >> LOGM, v = idx & MASK;
                const int ph = (u * m + v * n) & MASK;
                val += car[it] * twc[ph] - cai[it] * tws[ph];
            }
        }
        for (int off = gs >> 1; off >= 1; off >>= 1) val += __shfl_xor(val, off);
        val *= g;  // the recorded values are R[u,v]; alpha = gamma R[u,v] / W0
        if (sub == 0 && H.lost[px]) {
            const int y = d.x + py, x = d.y + pxx;
            const int64_t q = (int64_t)y * J.W + x;
            J.recon[q] = val;
            if (y >= J.cy0 && y < J.cy1 && x >= J.cx0 && x < J.cx1)
                J.out[(int64_t)(J.oy + y) * J.out_pitch + (J.ox + x)] = (float)val;
        }
    }
    // every wave's pixel stores complete before the barrier; the release
    // fence of the publishing thread after it then covers them (one cache
    // write-back per block instead of one per wave)
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();  // also: the coefficient list is read before the next block reuses the area
}

// ---------------------------------------------------------------------------
// dependency wait: every earlier block whose lost pixels meet this block's
// window, or whose window meets this block's lost pixels
// ---------------------------------------------------------------------------
template <int NT>
__device__ void wait_predecessors(const LaunchArgs& a, const JobDev& J, int blk) {
    const int4 d = uniform_load(J.desc + blk);
    const int4 lb = uniform_load(J.lbox + blk);
    const ClassDev& Cj = a.cls[d.z];
    const int Bm = a.Bmin;
    // fine cells that may hold an interacting block
    const int ry0 = d.x - a.reach, rx0 = d.y - a.reach;
    const int ry1 = d.x + Cj.B + a.reach, rx1 = d.y + Cj.B + a.reach;
    const int fy0 = max(0, ry0 >= 0 ? ry0 / Bm : 0), fx0 = max(0, rx0 >= 0 ? rx0 / Bm : 0);
    const int fy1 = min(J.fh - 1, (ry1 - 1) / Bm), fx1 = min(J.fw - 1, (rx1 - 1) / Bm);
    const int nw = fx1 - fx0 + 1;
    const int ncell = (fy1 - fy0 + 1) * nw;
    // window of j
    const int jwy0 = d.x - Cj.b, jwx0 = d.y - Cj.b;
    const int jwy1 = d.x + Cj.B + Cj.b, jwx1 = d.y + Cj.B + Cj.b;
    for (int c = threadIdx.x; c < ncell; c += NT) {
        const int fy = fy0 + c / nw, fx = fx0 + c % nw;
        const int i = J.owner[fy * J.fw + fx];
        if (i < 0 || i >= blk) continue;
        const int4 di = J.desc[i];
        // count each neighbour once: at its first cell inside the scanned range
        const int iy = max(fy0, di.x / Bm), ix = max(fx0, di.y / Bm);
        if (iy != fy || ix != fx) continue;
        const int4 li = J.lbox[i];
        const ClassDev& Ci = a.cls[di.z];
        const bool e1 = boxes_meet(li.x, li.y, li.z, li.w, jwy0, jwx0, jwy1, jwx1);
        const bool e2 = boxes_meet(lb.x, lb.y, lb.z, lb.w, di.x - Ci.b, di.y - Ci.b, di.x + Ci.B + Ci.b,
                                   di.y + Ci.B + Ci.b);
        if (!(e1 || e2)) continue;
        if (ld_flag(&J.done[i]) == 0) {
            const uint64_t t0 = wall_clock64();
            while (ld_flag(&J.done[i]) == 0) {
                __builtin_amdgcn_s_sleep(2);
                if ((int64_t)(wall_clock64() - t0) > a.wait_limit) {
                    atomicOr(a.error, 1);
                    break;
                }
            }
        }
    }
    // the flags read above were all set: one acquire fence (it invalidates
    // the CU's and the L2's stale lines for every wave of the workgroup),
    // ordered before the other waves' loads by the barrier after it
    __syncthreads();
    if (threadIdx.x < 64) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __syncthreads();
}

// ---------------------------------------------------------------------------
// block kernel: tickets in dispatch order; with counter != null the grid is
// persistent and workgroups draw tickets until none is left
// ---------------------------------------------------------------------------
// WIDE: the launch holds M = 64 blocks (the shared area is sized for them and
// each block branches on its window size).
template <int NW, int PREC, bool WIDE>
// Occupancy (the second bound counts waves per SIMD): the 4-wave 32 x 32
// kernels hold five blocks per CU (96 VGPRs); the FP64 kernel of launches
// with 64 x 64 windows two (eight waves each, so four per SIMD: 128 VGPRs;
// 73 KB of LDS each).
__global__ void __launch_bounds__(64 * NW, (NW == 4 && !WIDE) ? 5 : (WIDE && PREC == 0) ? 4 : 1)
    k_fse_blocks(LaunchArgs a, int ticket_base) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    SharedHead& H = *reinterpret_cast<SharedHead*>(smem_raw);
    double* buf = reinterpret_cast<double*>(smem_raw + sizeof(SharedHead));
    const int t = threadIdx.x;
    if (t < 32) {
        H.twc32[t] = a.tw32[t];
        H.tws32[t] = a.tw32[32 + t];
    }
    double* tw64 = nullptr;
    if constexpr (WIDE) {
        Shared64& S = *reinterpret_cast<Shared64*>(smem_raw);
        tw64 = S.tw64;
        if (t < 128) tw64[t] = a.tw64[t];
        buf = S.buf;
    }
    for (;;) {
        if (t == 0) {
            int tk;
            if (a.counter)
                tk = __hip_atomic_fetch_add(a.counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else
                tk = ticket_base + blockIdx.x;
            if (tk < a.n_tickets) {
                const int2 tkt = a.tickets[tk];
                H.job = tkt.x;
                H.blk = tkt.y;
            } else {
                H.job = -1;
                H.blk = -1;
            }
        }
        __syncthreads();
        const int job = __builtin_amdgcn_readfirstlane(H.job), blk = __builtin_amdgcn_readfirstlane(H.blk);
        if (job < 0) break;
        const JobDev J = uniform_load(a.jobs + job);
        if constexpr (WIDE) {
            // 64 x 64 windows on all waves; 32 x 32 windows on four of them
            if (a.cls[J.desc[blk].z].M == 64)
                process_block<64, NW, NW, PREC>(a, J, blk, H, buf, tw64);
            else
                process_block<32, 4, NW, PREC>(a, J, blk, H, buf, tw64);
        } else {
            process_block<32, NW, NW, PREC>(a, J, blk, H, buf, tw64);
        }
        // process_block ends with a barrier after every wave's stores: thread
        // 0 publishes the block, then takes the next ticket (the other waves
        // read the ticket's LDS slots only after the barrier at the top)
        if (t == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_store(&J.done[blk], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (!a.counter) break;
    }
}

static const void* kernel_for(int nw, int prec, bool wide) {
    if (wide) {  // launches with 64 x 64 windows run eight waves per workgroup
        if (prec == kPrecF32) return (const void*)k_fse_blocks<kWideWaves, 1, true>;
        if (prec == kPrecBF16x3) return (const void*)k_fse_blocks<kWideWaves, 2, true>;
        return (const void*)k_fse_blocks<kWideWaves, 0, true>;
    }
#define FSE_K(N, P) (const void*)k_fse_blocks<N, P, false>
    if (prec == kPrecF32) return nw == 1 ? FSE_K(1, 1) : nw == 2 ? FSE_K(2, 1) : FSE_K(4, 1);
    if (prec == kPrecBF16x3) return nw == 1 ? FSE_K(1, 2) : nw == 2 ? FSE_K(2, 2) : FSE_K(4, 2);
    return nw == 1 ? FSE_K(1, 0) : nw == 2 ? FSE_K(2, 0) : FSE_K(4, 0);
#undef FSE_K
}

size_t shared_bytes_blocks(bool wide) { return wide ? sizeof(Shared64) : sizeof(Shared32); }

int persistent_grid(int nw, int prec, bool wide) {
    int dev = 0, cus = 0, per_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const void* k = kernel_for(nw, prec, wide);
    const int nthreads = 64 * (wide ? kWideWaves : nw);
    const int lds = (int)shared_bytes_blocks(wide);
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, nthreads, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return std::max(1, cus) * per_cu;
}

hipError_t launch_blocks_at(const LaunchArgs& a, int nw, int prec, bool wide, int grid, int ticket_base,
                            hipStream_t st) {
    const void* k = kernel_for(nw, prec, wide);
    const int nthreads = 64 * (wide ? kWideWaves : nw);
    const int lds = (int)shared_bytes_blocks(wide);
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    void* args[] = {(void*)&a, (void*)&ticket_base};
    return hipLaunchKernel(k, dim3(grid), dim3(nthreads), args, lds, st);
}

}  // namespace fse
