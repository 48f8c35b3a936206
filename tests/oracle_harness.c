/* The FP64 oracle (oracle/fse_oracle.c) from a plain C driver, for a CPU test
 * that builds both with the address and undefined-behaviour sanitizers:
 *   oracle_harness IMGFILE MASKFILE OUTFILE W H B1 b1 K1 [B2 b2 K2 [B3 b3 K3]]
 * IMGFILE holds W*H doubles, MASKFILE W*H bytes (1 = lost); OUTFILE receives
 * the W*H doubles of the extrapolated image (rho 0.8, gamma 0.5, delta 0.5). */
#include <stdio.h>
#include <stdlib.h>

int fse_oracle_image(const double* img, const unsigned char* mask, int W, int H, const int* classes,
                     int n_classes, double rho, double gamma, double delta, const int* order,
                     double* out, int Kmax, int* trace_sel, double* trace_e, int* trace_i,
                     double* trace_a, double* trace_w0);

static int slurp(const char* path, void* dst, size_t bytes) {
    FILE* f = fopen(path, "rb");
    if (!f) return -1;
    const size_t got = fread(dst, 1, bytes, f);
    fclose(f);
    return got == bytes ? 0 : -1;
}

int main(int argc, char** argv) {
    if (argc < 9 || (argc - 6) % 3 != 0) {
        fprintf(stderr, "usage: oracle_harness IMG MASK OUT W H B1 b1 K1 [...]\n");
        return 2;
    }
    const int W = atoi(argv[4]), H = atoi(argv[5]);
    const int nc = (argc - 6) / 3;
    int classes[9];
    int kmax = 1;
    for (int i = 0; i < 3 * nc; ++i) classes[i] = atoi(argv[6 + i]);
    for (int c = 0; c < nc; ++c)
        if (classes[3 * c + 2] > kmax) kmax = classes[3 * c + 2];
    const size_t n = (size_t)W * H;
    double* img = (double*)malloc(n * sizeof(double));
    double* out = (double*)calloc(n, sizeof(double));
    unsigned char* mask = (unsigned char*)malloc(n);
    if (!img || !out || !mask || slurp(argv[1], img, n * sizeof(double)) || slurp(argv[2], mask, n)) return 2;
    const int rc = fse_oracle_image(img, mask, W, H, classes, nc, 0.8, 0.5, 0.5, NULL, out, kmax, NULL, NULL,
                                    NULL, NULL, NULL);
    if (rc < 0) return 3;
    FILE* f = fopen(argv[3], "wb");
    if (!f || fwrite(out, sizeof(double), n, f) != n) return 4;
    fclose(f);
    free(img);
    free(out);
    free(mask);
    return 0;
}
