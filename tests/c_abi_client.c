/*
 * A plain C client of libfse: device buffers from hipMalloc, no Python.
 *
 * A constant image is the closed-form case of the method: every step selects
 * the DC basis function, and after K steps with gamma = 1/2 the model holds
 * c (1 - 2^-K), so every lost pixel comes back as c (to float rounding) while
 * every known pixel is copied.  Checked for the whole image and for the tile
 * framework.  Exit status 0 on success.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "fse.h"

#define CHECK_HIP(x)                                                   \
    do {                                                               \
        hipError_t e_ = (x);                                           \
        if (e_ != hipSuccess) {                                        \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));    \
            return 2;                                                  \
        }                                                              \
    } while (0)

static int run(int tiled, int W, int H, const float* h_img, const uint8_t* h_mask, float c) {
    const size_t n = (size_t)W * H;
    float *d_img = NULL, *d_out = NULL;
    uint8_t* d_mask = NULL;
    CHECK_HIP(hipMalloc((void**)&d_img, n * sizeof(float)));
    CHECK_HIP(hipMalloc((void**)&d_out, n * sizeof(float)));
    CHECK_HIP(hipMalloc((void**)&d_mask, n));
    CHECK_HIP(hipMemcpy(d_img, h_img, n * sizeof(float), hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d_mask, h_mask, n, hipMemcpyHostToDevice));

    fse_params_t p;
    if (fse_params_default(&p) != FSE_OK) return 3;
    if (tiled) {
        p.tiling = FSE_TILED;
        p.n_tiles = 6;
        p.overlap = 16;
        p.align = 4;
    }
    fse_image_t im = {d_img, W, H, W};
    fse_mask_t mk = {d_mask, W, H, W};
    fse_image_t out = {d_out, W, H, W};
    fse_status_t s = fse_extrapolate(&im, &mk, &p, &out, NULL);
    if (s != FSE_OK) {
        fprintf(stderr, "fse_extrapolate: %s\n", fse_status_string(s));
        return 4;
    }
    fse_run_stats_t st;
    if (fse_last_stats(&st) != FSE_OK || st.device_error) return 5;

    float* h_out = (float*)malloc(n * sizeof(float));
    CHECK_HIP(hipMemcpy(h_out, d_out, n * sizeof(float), hipMemcpyDeviceToHost));
    double max_lost = 0.0;
    size_t lost = 0;
    for (size_t i = 0; i < n; ++i) {
        if (h_mask[i]) {
            const double e = fabs((double)h_out[i] - c);
            if (!(e <= max_lost)) max_lost = e; /* also catches NaN */
            ++lost;
        } else if (h_out[i] != h_img[i]) {
            fprintf(stderr, "known pixel %zu changed\n", i);
            return 6;
        }
    }
    printf("%s: %zu lost pixels, %lld blocks, %lld jobs, max |out - c| = %.3g, kernel %.3f ms\n",
           tiled ? "tiled" : "whole", lost, (long long)st.n_blocks, (long long)st.n_jobs, max_lost, st.kernel_ms);
    free(h_out);
    (void)hipFree(d_img);
    (void)hipFree(d_out);
    (void)hipFree(d_mask);
    return max_lost <= 1e-3 ? 0 : 7;
}

int main(void) {
    const int W = 150, H = 93;
    const float c = 117.25f;
    float* img = (float*)malloc((size_t)W * H * sizeof(float));
    uint8_t* mask = (uint8_t*)calloc((size_t)W * H, 1);
    for (int i = 0; i < W * H; ++i) img[i] = c;
    /* every third 4x4 block of the grid lost, plus a few isolated pixels */
    for (int by = 0; by < H / 4; ++by)
        for (int bx = 0; bx < W / 4; ++bx)
            if ((by * 7 + bx) % 3 == 0)
                for (int y = 0; y < 4; ++y)
                    for (int x = 0; x < 4; ++x) mask[(by * 4 + y) * W + bx * 4 + x] = 1;
    for (int i = 5; i < W * H; i += 97) mask[i] = 1;
    int rc = run(0, W, H, img, mask, c);
    if (rc == 0) rc = run(1, W, H, img, mask, c);
    free(img);
    free(mask);
    if (fse_release() != FSE_OK && rc == 0) rc = 8;
    return rc;
}
