/*
 * fse_oracle.c -- plain FP64 CPU reference of Frequency Selective Extrapolation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU baseline of the
 * benchmark do.  It shares no code, header, table or constant with the HIP
 * path.
 *
 * What it computes (Sec. II of the paper, the block model it parallelises):
 * the image is cut into small processing blocks; the lost pixels of each block
 * are replaced by a sparse model -- a weighted superposition of 2-D DFT basis
 * functions -- fitted to the known and already reconstructed pixels of a
 * support window around the block.  The fit is greedy: in each of K steps the
 * basis function whose weighted projection removes most residual energy is
 * chosen and a fraction gamma of that projection is added to the model
 * (the orthogonality-deficiency compensation).  The paper gives the method in
 * prose only; the formulas below follow the standard form of the complex FSE
 * and every reading that the paper leaves open is listed in the design notes
 * as R1..R16.
 *
 * Notation (window of M x M pixels, m = row, n = column, 0-based):
 *   w[m,n]   weight: rho^dist for known pixels, delta*rho^dist for pixels
 *            reconstructed by earlier blocks, 0 for lost or off-image pixels;
 *            dist = distance of (m,n) from the window centre ((M-1)/2,(M-1)/2)
 *   s[m,n]   pixel value where w > 0, else 0 (lost values are never read)
 *   W0       sum of w
 *   R[k,l]   weighted residual spectrum  sum_{m,n} w s e^{-2 pi i (k m + l n)/M}
 *   Wsp[k,l] weight spectrum             sum_{m,n} w   e^{-2 pi i (k m + l n)/M}
 *   step:    (u,v) = argmax |R|^2 (ties -> smallest k*M+l)
 *            alpha = gamma * R[u,v] / W0,   c[u,v] += alpha
 *            R[k,l] -= alpha * Wsp[(k-u) mod M, (l-v) mod M]
 *   model:   g[m,n] = sum over steps of alpha e^{+2 pi i (u m + v n)/M};
 *            the lost pixels of the block receive Re g.
 *
 * Blocks: the largest configured block class whose aligned square is entirely
 * lost forms one block; remaining lost pixels go to the aligned cells of the
 * smallest class.  Blocks are processed in raster order of their top-left
 * corner unless an explicit order is passed (used to check that a
 * dependency-respecting order gives the same result).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ST_KNOWN 0
#define ST_LOST 1
#define ST_RECON 2
#define ST_OUT 3

#define TOPN 4

static const double TWO_PI = 6.283185307179586476925286766559;

/* e^{-2 pi i p / M} for p = 0..M-1; every phase used below is reduced mod M
 * in integer arithmetic first, so each twiddle is one correctly evaluated
 * cos/sin pair. */
static void twiddles(int M, double* c, double* s) {
    for (int p = 0; p < M; ++p) {
        c[p] = cos(TWO_PI * (double)p / (double)M);
        s[p] = -sin(TWO_PI * (double)p / (double)M);
    }
}

/* 2-D DFT of a complex M x M array written as the matrix product F X F
 * (F[k,m] = e^{-2 pi i k m / M} is symmetric):  first T = F X, then Y = T F. */
static void dft2(int M, const double* xr, const double* xi, double* yr, double* yi,
                 const double* tc, const double* ts) {
    double* trr = (double*)malloc(sizeof(double) * M * M);
    double* tii = (double*)malloc(sizeof(double) * M * M);
    for (int k = 0; k < M; ++k)
        for (int n = 0; n < M; ++n) {
            double ar = 0.0, ai = 0.0;
            for (int m = 0; m < M; ++m) {
                int p = (k * m) % M;
                double fr = tc[p], fi = ts[p];
                double vr = xr[m * M + n], vi = xi ? xi[m * M + n] : 0.0;
                ar += fr * vr - fi * vi;
                ai += fr * vi + fi * vr;
            }
            trr[k * M + n] = ar;
            tii[k * M + n] = ai;
        }
    for (int k = 0; k < M; ++k)
        for (int l = 0; l < M; ++l) {
            double ar = 0.0, ai = 0.0;
            for (int n = 0; n < M; ++n) {
                int p = (n * l) % M;
                double fr = tc[p], fi = ts[p];
                double vr = trr[k * M + n], vi = tii[k * M + n];
                ar += vr * fr - vi * fi;
                ai += vr * fi + vi * fr;
            }
            yr[k * M + l] = ar;
            yi[k * M + l] = ai;
        }
    free(trr);
    free(tii);
}

/*
 * One block: the greedy sparse fit on one support window.
 *   s_re/s_im : window values (s_im may be NULL for a real window), M*M
 *   w         : weights, M*M (0 marks unusable pixels; their s is ignored)
 *   K, gamma  : number of steps and compensation factor
 * outputs (each may be NULL):
 *   sel[K]          chosen index u*M+v per step
 *   a_re/a_im[K]    alpha per step
 *   R_hist          (K+1) * 2 * M*M doubles: R (re block, im block) before
 *                   step 1 and after every step
 *   e_top[K*TOPN], i_top[K*TOPN]: the TOPN largest energies |R|^2 before each
 *                   step, descending, ties by smallest index, and their indices
 * returns W0 (0 when no pixel carries weight; then no step is taken).
 */
double fse_oracle_block(int M, const double* s_re, const double* s_im, const double* w, int K,
                        double gamma, int* sel, double* a_re, double* a_im, double* R_hist,
                        double* e_top, int* i_top) {
    const int MM = M * M;
    double* tc = (double*)malloc(sizeof(double) * M);
    double* ts = (double*)malloc(sizeof(double) * M);
    twiddles(M, tc, ts);

    double W0 = 0.0;
    for (int q = 0; q < MM; ++q) W0 += w[q];

    double* xr = (double*)calloc(MM, sizeof(double));
    double* xi = (double*)calloc(MM, sizeof(double));
    for (int q = 0; q < MM; ++q) {
        if (w[q] > 0.0) {
            xr[q] = w[q] * s_re[q];
            xi[q] = s_im ? w[q] * s_im[q] : 0.0;
        }
    }
    double* Rr = (double*)malloc(sizeof(double) * MM);
    double* Ri = (double*)malloc(sizeof(double) * MM);
    double* Wr = (double*)malloc(sizeof(double) * MM);
    double* Wi = (double*)malloc(sizeof(double) * MM);
    dft2(M, xr, xi, Rr, Ri, tc, ts);
    dft2(M, w, NULL, Wr, Wi, tc, ts);
    if (R_hist) {
        memcpy(R_hist, Rr, sizeof(double) * MM);
        memcpy(R_hist + MM, Ri, sizeof(double) * MM);
    }

    double* e = (double*)malloc(sizeof(double) * MM);
    for (int it = 0; it < K && W0 > 0.0; ++it) {
        for (int q = 0; q < MM; ++q) e[q] = Rr[q] * Rr[q] + Ri[q] * Ri[q];
        int best = 0;
        for (int q = 1; q < MM; ++q)
            if (e[q] > e[best]) best = q; /* strict: the first index wins ties */
        if (e_top && i_top) {
            /* TOPN largest, selection by repeated scans (plain, small TOPN) */
            for (int t = 0; t < TOPN; ++t) {
                int arg = -1;
                for (int q = 0; q < MM; ++q) {
                    int used = 0;
                    for (int r = 0; r < t; ++r) used |= (i_top[it * TOPN + r] == q);
                    if (used) continue;
                    if (arg < 0 || e[q] > e[arg]) arg = q;
                }
                i_top[it * TOPN + t] = arg;
                e_top[it * TOPN + t] = arg >= 0 ? e[arg] : 0.0;
            }
        }
        int u = best / M, v = best % M;
        double ar = gamma * Rr[best] / W0;
        double ai = gamma * Ri[best] / W0;
        if (sel) sel[it] = best;
        if (a_re) a_re[it] = ar;
        if (a_im) a_im[it] = ai;
        for (int k = 0; k < M; ++k)
            for (int l = 0; l < M; ++l) {
                int q = k * M + l;
                int sh = ((k - u + M) % M) * M + ((l - v + M) % M);
                Rr[q] -= ar * Wr[sh] - ai * Wi[sh];
                Ri[q] -= ar * Wi[sh] + ai * Wr[sh];
            }
        if (R_hist) {
            memcpy(R_hist + (size_t)(it + 1) * 2 * MM, Rr, sizeof(double) * MM);
            memcpy(R_hist + (size_t)(it + 1) * 2 * MM + MM, Ri, sizeof(double) * MM);
        }
    }
    free(e);
    free(xr);
    free(xi);
    free(Rr);
    free(Ri);
    free(Wr);
    free(Wi);
    free(tc);
    free(ts);
    return W0;
}

/* Model value at window position (m,n): sum_nu alpha_nu e^{+2 pi i (u m + v n)/M}. */
static void synth_at(int M, int K, const int* sel, const double* a_re, const double* a_im, int m,
                     int n, double* gr, double* gi) {
    double sr = 0.0, si = 0.0;
    for (int it = 0; it < K; ++it) {
        int u = sel[it] / M, v = sel[it] % M;
        int p = (u * m + v * n) % M;
        double c = cos(TWO_PI * (double)p / (double)M);
        double s = sin(TWO_PI * (double)p / (double)M);
        sr += a_re[it] * c - a_im[it] * s;
        si += a_re[it] * s + a_im[it] * c;
    }
    *gr = sr;
    *gi = si;
}

/*
 * Processing blocks from the mask.  classes: n_classes triples (B, border, K),
 * largest B first.  Every class but the last takes aligned B x B squares that
 * are entirely lost and not yet taken; the last class takes each aligned cell
 * (clipped at the image edge) that still holds a lost pixel.  The blocks are
 * written in raster order of (y0, x0); owner (H*W, may be NULL) receives the
 * block index of every lost pixel and -1 elsewhere.
 * Returns the number of blocks, or -(needed) when max_blocks is too small.
 */
int fse_oracle_plan(const unsigned char* mask, int W, int H, const int* classes, int n_classes,
                    int* blk_y, int* blk_x, int* blk_cls, int max_blocks, int* owner) {
    int* own = (int*)malloc(sizeof(int) * (size_t)W * H);
    for (size_t q = 0; q < (size_t)W * H; ++q) own[q] = -1;
    /* provisional ids: record blocks in discovery order, sort afterwards */
    int cap = 1024, n = 0;
    int* by = (int*)malloc(sizeof(int) * cap);
    int* bx = (int*)malloc(sizeof(int) * cap);
    int* bc = (int*)malloc(sizeof(int) * cap);
    for (int c = 0; c < n_classes; ++c) {
        int B = classes[3 * c];
        int last = (c == n_classes - 1);
        for (int y0 = 0; y0 < H; y0 += B)
            for (int x0 = 0; x0 < W; x0 += B) {
                int take;
                if (last) {
                    take = 0;
                    for (int y = y0; y < y0 + B && y < H; ++y)
                        for (int x = x0; x < x0 + B && x < W; ++x)
                            if (mask[(size_t)y * W + x] && own[(size_t)y * W + x] < 0) take = 1;
                } else {
                    take = (y0 + B <= H) && (x0 + B <= W);
                    for (int y = y0; take && y < y0 + B; ++y)
                        for (int x = x0; x < x0 + B; ++x)
                            if (!mask[(size_t)y * W + x] || own[(size_t)y * W + x] >= 0) {
                                take = 0;
                                break;
                            }
                }
                if (!take) continue;
                if (n == cap) {
                    cap *= 2;
                    by = (int*)realloc(by, sizeof(int) * cap);
                    bx = (int*)realloc(bx, sizeof(int) * cap);
                    bc = (int*)realloc(bc, sizeof(int) * cap);
                }
                for (int y = y0; y < y0 + B && y < H; ++y)
                    for (int x = x0; x < x0 + B && x < W; ++x)
                        if (mask[(size_t)y * W + x] && own[(size_t)y * W + x] < 0)
                            own[(size_t)y * W + x] = n;
                by[n] = y0;
                bx[n] = x0;
                bc[n] = c;
                ++n;
            }
    }
    /* raster order of (y0, x0): plain insertion into a position array */
    int* pos = (int*)malloc(sizeof(int) * (n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) pos[i] = i;
    /* simple merge-free sort: counting by row then stable by column would also
       do; a plain comparison sort keeps it obvious */
    for (int i = 1; i < n; ++i) {
        int key = pos[i], j = i - 1;
        while (j >= 0 && (by[pos[j]] > by[key] || (by[pos[j]] == by[key] && bx[pos[j]] > bx[key]))) {
            pos[j + 1] = pos[j];
            --j;
        }
        pos[j + 1] = key;
    }
    int ret = n;
    if (n > max_blocks) {
        ret = -n;
    } else {
        int* rank = (int*)malloc(sizeof(int) * (n > 0 ? n : 1));
        for (int i = 0; i < n; ++i) {
            blk_y[i] = by[pos[i]];
            blk_x[i] = bx[pos[i]];
            blk_cls[i] = bc[pos[i]];
            rank[pos[i]] = i;
        }
        if (owner)
            for (size_t q = 0; q < (size_t)W * H; ++q) owner[q] = own[q] >= 0 ? rank[own[q]] : -1;
        free(rank);
    }
    free(pos);
    free(by);
    free(bx);
    free(bc);
    free(own);
    return ret;
}

/*
 * Support window of one block from an image state: status per pixel
 * (0 known, 1 lost, 2 reconstructed) and the current values.  Off-image
 * pixels carry no weight.  w and s are M*M.
 */
static void window_of(const double* val, const unsigned char* status, int W, int H, int wy, int wx, int M,
                      double rho, double delta, double* w, double* s) {
    double ctr = 0.5 * (double)(M - 1);
    for (int m = 0; m < M; ++m)
        for (int n = 0; n < M; ++n) {
            int y = wy + m, x = wx + n;
            int st = (y < 0 || y >= H || x < 0 || x >= W) ? ST_OUT : status[(size_t)y * W + x];
            double dist = sqrt((m - ctr) * (m - ctr) + (n - ctr) * (n - ctr));
            double wt = 0.0;
            if (st == ST_KNOWN) wt = pow(rho, dist);
            else if (st == ST_RECON) wt = delta * pow(rho, dist);
            w[m * M + n] = wt;
            s[m * M + n] = wt > 0.0 ? val[(size_t)y * W + x] : 0.0;
        }
}

/*
 * One block in isolation: the block of edge B with top-left (y0, x0) and
 * border b is extrapolated from the given image state (val, status as in
 * window_of).  out_vals[B*B] receives Re of the model at every pixel of the
 * block (row-major, pixels outside the image left untouched); sel[K] (may be
 * NULL) the chosen indices.  Returns W0.
 */
double fse_oracle_one_block(const double* val, const unsigned char* status, int W, int H, int y0, int x0,
                            int B, int b, int K, double rho, double gamma, double delta, double* out_vals,
                            int* sel_out) {
    int M = B + 2 * b;
    double* w = (double*)calloc((size_t)M * M, sizeof(double));
    double* s = (double*)calloc((size_t)M * M, sizeof(double));
    int* sel = (int*)malloc(sizeof(int) * (K > 0 ? K : 1));
    double* ar = (double*)malloc(sizeof(double) * (K > 0 ? K : 1));
    double* ai = (double*)malloc(sizeof(double) * (K > 0 ? K : 1));
    window_of(val, status, W, H, y0 - b, x0 - b, M, rho, delta, w, s);
    double W0 = fse_oracle_block(M, s, NULL, w, K, gamma, sel, ar, ai, NULL, NULL, NULL);
    for (int py = 0; py < B; ++py)
        for (int px = 0; px < B; ++px) {
            double gr = 0.0, gi = 0.0;
            if (W0 > 0.0) synth_at(M, K, sel, ar, ai, b + py, b + px, &gr, &gi);
            out_vals[py * B + px] = gr;
        }
    if (sel_out)
        for (int it = 0; it < K; ++it) sel_out[it] = W0 > 0.0 ? sel[it] : -1;
    free(w);
    free(s);
    free(sel);
    free(ar);
    free(ai);
    return W0;
}

/*
 * Optimised processing order (Sec. II: the order follows the shape and the
 * distribution of the lost pixels, so that large lost areas close from their
 * margins towards their centre).  The rule itself is in work the paper cites
 * and does not print; the reading implemented here (R17):
 *
 *   Each step processes, among the blocks not yet processed, the block whose
 *   support window currently offers the largest share of usable weight: the
 *   sum of its window weights under the current pixel statuses (R7: rho^dist
 *   for known pixels, delta rho^dist for reconstructed ones, 0 for lost or
 *   off-image pixels), divided by that sum for a window of its class whose
 *   pixels are all known.  Equal shares go to the block that comes first in
 *   raster order.
 *
 * The weights enter as integers, q = round(2^30 rho^dist) and
 * qr = round(2^30 delta rho^dist), so every sum is exact and every tie is a
 * true tie; shares are compared by cross-multiplication in 128-bit integers.
 * The order depends on the mask alone.
 *
 * Plain implementation: after each step the share of every remaining block
 * whose window meets the processed block is summed again over its whole
 * window from the status map, and the next block is found by a scan over all
 * blocks.  order[k] receives the raster index of the k-th block processed
 * (order has room for every block).  Returns the number of blocks, or -1.
 */
typedef unsigned __int128 u128;

static long long q_weight(double rho, double delta, int M, int m, int n, int recon) {
    double dm = m - (M - 1) / 2.0, dn = n - (M - 1) / 2.0; /* from the window centre */
    double wt = pow(rho, sqrt(dm * dm + dn * dn));
    if (recon) wt = delta * wt;
    return llround(ldexp(wt, 30));
}

static long long window_share_sum(const unsigned char* status, int W, int H, int wy, int wx, int M,
                                  const long long* qk, const long long* qr) {
    long long sum = 0;
    for (int m = 0; m < M; ++m)
        for (int n = 0; n < M; ++n) {
            int y = wy + m, x = wx + n;
            if (y < 0 || y >= H || x < 0 || x >= W) continue;
            unsigned char st = status[(size_t)y * W + x];
            if (st == ST_KNOWN) sum += qk[m * M + n];
            else if (st == ST_RECON) sum += qr[m * M + n];
        }
    return sum;
}

int fse_oracle_priority_order(const unsigned char* mask, int W, int H, const int* classes, int n_classes,
                              double rho, double delta, int* order) {
    if (W <= 0 || H <= 0 || n_classes <= 0 || n_classes > 8 || !order) return -1;
    int nb = fse_oracle_plan(mask, W, H, classes, n_classes, NULL, NULL, NULL, 0, NULL);
    int nmax = nb < 0 ? -nb : nb;
    int* by = (int*)malloc(sizeof(int) * (nmax + 1));
    int* bx = (int*)malloc(sizeof(int) * (nmax + 1));
    int* bc = (int*)malloc(sizeof(int) * (nmax + 1));
    int* owner = (int*)malloc(sizeof(int) * (size_t)W * H);
    nb = fse_oracle_plan(mask, W, H, classes, n_classes, by, bx, bc, nmax, owner);

    long long* qk[8];
    long long* qr[8];
    long long full[8];
    for (int c = 0; c < n_classes; ++c) {
        int M = classes[3 * c] + 2 * classes[3 * c + 1];
        qk[c] = (long long*)malloc(sizeof(long long) * M * M);
        qr[c] = (long long*)malloc(sizeof(long long) * M * M);
        full[c] = 0;
        for (int m = 0; m < M; ++m)
            for (int n = 0; n < M; ++n) {
                qk[c][m * M + n] = q_weight(rho, delta, M, m, n, 0);
                qr[c][m * M + n] = q_weight(rho, delta, M, m, n, 1);
                full[c] += qk[c][m * M + n];
            }
    }
    unsigned char* status = (unsigned char*)malloc((size_t)W * H);
    for (size_t q = 0; q < (size_t)W * H; ++q) status[q] = mask[q] ? ST_LOST : ST_KNOWN;
    long long* share = (long long*)malloc(sizeof(long long) * (nmax + 1));
    unsigned char* done = (unsigned char*)calloc(nmax + 1, 1);
    for (int i = 0; i < nb; ++i) {
        int c = bc[i], B = classes[3 * c], b = classes[3 * c + 1];
        share[i] = window_share_sum(status, W, H, by[i] - b, bx[i] - b, B + 2 * b, qk[c], qr[c]);
    }
    for (int k = 0; k < nb; ++k) {
        int best = -1;
        for (int i = 0; i < nb; ++i) {
            if (done[i]) continue;
            /* share[i] / full[c_i] > share[best] / full[c_best], strictly:
               the raster-earlier block keeps a tie */
            if (best < 0 || (u128)share[i] * (u128)full[bc[best]] > (u128)share[best] * (u128)full[bc[i]])
                best = i;
        }
        order[k] = best;
        done[best] = 1;
        int cb = bc[best], Bb = classes[3 * cb];
        for (int y = by[best]; y < by[best] + Bb && y < H; ++y)
            for (int x = bx[best]; x < bx[best] + Bb && x < W; ++x)
                if (owner[(size_t)y * W + x] == best) status[(size_t)y * W + x] = ST_RECON;
        for (int i = 0; i < nb; ++i) {
            if (done[i]) continue;
            int c = bc[i], B = classes[3 * c], b = classes[3 * c + 1];
            int wy = by[i] - b, wx = bx[i] - b, M = B + 2 * b;
            if (wy < by[best] + Bb && by[best] < wy + M && wx < bx[best] + Bb && bx[best] < wx + M)
                share[i] = window_share_sum(status, W, H, wy, wx, M, qk[c], qr[c]);
        }
    }
    for (int c = 0; c < n_classes; ++c) {
        free(qk[c]);
        free(qr[c]);
    }
    free(status);
    free(share);
    free(done);
    free(owner);
    free(by);
    free(bx);
    free(bc);
    return nb;
}

/*
 * One block of the whole-image process: its window from the current state,
 * the greedy fit, and the model written into the lost pixels it owns (their
 * status becomes reconstructed).  cls = (B, border, K).  sel/ar/ai receive
 * the K steps; et/itp (may be NULL) the top energies.  Returns W0.
 */
static double run_block(int bi, int y0, int x0, const int* cls, const int* owner, double* out,
                        unsigned char* status, int W, int H, double rho, double gamma, double delta, int* sel,
                        double* ar, double* ai, double* et, int* itp) {
    int B = cls[0], b = cls[1], K = cls[2];
    int M = B + 2 * b;
    int wy = y0 - b, wx = x0 - b;
    double* w = (double*)calloc((size_t)M * M, sizeof(double));
    double* s = (double*)calloc((size_t)M * M, sizeof(double));
    window_of(out, status, W, H, wy, wx, M, rho, delta, w, s);
    double W0 = fse_oracle_block(M, s, NULL, w, K, gamma, sel, ar, ai, NULL, et, itp);
    for (int m = 0; m < M; ++m)
        for (int n = 0; n < M; ++n) {
            int y = wy + m, x = wx + n;
            if (y < 0 || y >= H || x < 0 || x >= W) continue;
            size_t q = (size_t)y * W + x;
            if (owner[q] != bi) continue;
            double gr = 0.0, gi = 0.0;
            if (W0 > 0.0) synth_at(M, K, sel, ar, ai, m, n, &gr, &gi);
            out[q] = gr;
            status[q] = ST_RECON;
        }
    free(w);
    free(s);
    return W0;
}

/*
 * Whole image.  img: H*W values (row-major).  mask: 1 = lost.  out: H*W,
 * receives img with every lost pixel replaced.  order (may be NULL): a
 * permutation of 0..n_blocks-1 giving the processing order by raster index.
 * Trace buffers (may be NULL): per raster block index b and step t,
 * trace_sel[b*Kmax+t], trace_e[(b*Kmax+t)*TOPN+r], trace_i[...] and the
 * coefficients trace_a[(b*Kmax+t)*2 + {0,1}]; trace_w0[b] = W0.
 * Returns the number of blocks, -1 on bad arguments, -2 when a block has no
 * weighted pixel (W0 = 0; its lost pixels are then set to 0).
 */
int fse_oracle_image(const double* img, const unsigned char* mask, int W, int H, const int* classes,
                     int n_classes, double rho, double gamma, double delta, const int* order,
                     double* out, int Kmax, int* trace_sel, double* trace_e, int* trace_i,
                     double* trace_a, double* trace_w0) {
    if (W <= 0 || H <= 0 || n_classes <= 0) return -1;
    int nmax = 0;
    int nb = fse_oracle_plan(mask, W, H, classes, n_classes, NULL, NULL, NULL, 0, NULL);
    nmax = nb < 0 ? -nb : nb;
    int* blk_y = (int*)malloc(sizeof(int) * (nmax + 1));
    int* blk_x = (int*)malloc(sizeof(int) * (nmax + 1));
    int* blk_c = (int*)malloc(sizeof(int) * (nmax + 1));
    int* owner = (int*)malloc(sizeof(int) * (size_t)W * H);
    nb = fse_oracle_plan(mask, W, H, classes, n_classes, blk_y, blk_x, blk_c, nmax, owner);

    unsigned char* status = (unsigned char*)malloc((size_t)W * H);
    for (size_t q = 0; q < (size_t)W * H; ++q) {
        out[q] = mask[q] ? 0.0 : img[q];
        status[q] = mask[q] ? ST_LOST : ST_KNOWN;
    }
    int rc = nb;
    for (int oi = 0; oi < nb; ++oi) {
        int bi = order ? order[oi] : oi;
        int c = blk_c[bi];
        int K = classes[3 * c + 2];
        int* sel = (int*)malloc(sizeof(int) * K);
        double* ar = (double*)malloc(sizeof(double) * K);
        double* ai = (double*)malloc(sizeof(double) * K);
        double* et = (double*)malloc(sizeof(double) * K * TOPN);
        int* itp = (int*)malloc(sizeof(int) * K * TOPN);
        double W0 = run_block(bi, blk_y[bi], blk_x[bi], classes + 3 * c, owner, out, status, W, H, rho, gamma,
                              delta, sel, ar, ai, trace_e ? et : NULL, trace_e ? itp : NULL);
        if (W0 <= 0.0) rc = -2;
        if (trace_w0) trace_w0[bi] = W0;
        for (int it = 0; it < K && it < Kmax; ++it) {
            size_t t = (size_t)bi * Kmax + it;
            if (trace_sel) trace_sel[t] = W0 > 0.0 ? sel[it] : -1;
            if (trace_a) {
                trace_a[2 * t] = W0 > 0.0 ? ar[it] : 0.0;
                trace_a[2 * t + 1] = W0 > 0.0 ? ai[it] : 0.0;
            }
            if (trace_e && trace_i)
                for (int r = 0; r < TOPN; ++r) {
                    trace_e[t * TOPN + r] = W0 > 0.0 ? et[it * TOPN + r] : 0.0;
                    trace_i[t * TOPN + r] = W0 > 0.0 ? itp[it * TOPN + r] : -1;
                }
        }
        free(sel);
        free(ar);
        free(ai);
        free(et);
        free(itp);
    }
    free(status);
    free(owner);
    free(blk_y);
    free(blk_x);
    free(blk_c);
    return rc;
}

/*
 * The raster-order extrapolation of fse_oracle_image, with the blocks of each
 * dependency level run in parallel on the host's cores (OpenMP).  A block
 * depends on an earlier block when either one owns a lost pixel inside the
 * other's support window (the window reads it, the owner writes it); a
 * block's level is one more than the largest level of the blocks it depends
 * on.  The blocks of one level neither read nor write each other's pixels,
 * so each block sees exactly the window it sees in raster order and the
 * output is bitwise the same.  *n_levels and *n_threads receive the number of
 * levels and the threads used.  Returns as fse_oracle_image.
 */
int fse_oracle_image_levels(const double* img, const unsigned char* mask, int W, int H, const int* classes,
                            int n_classes, double rho, double gamma, double delta, double* out, int* n_levels,
                            int* n_threads) {
    if (W <= 0 || H <= 0 || n_classes <= 0) return -1;
    int nb = fse_oracle_plan(mask, W, H, classes, n_classes, NULL, NULL, NULL, 0, NULL);
    int nmax = nb < 0 ? -nb : nb;
    int* blk_y = (int*)malloc(sizeof(int) * (nmax + 1));
    int* blk_x = (int*)malloc(sizeof(int) * (nmax + 1));
    int* blk_c = (int*)malloc(sizeof(int) * (nmax + 1));
    int* owner = (int*)malloc(sizeof(int) * (size_t)W * H);
    nb = fse_oracle_plan(mask, W, H, classes, n_classes, blk_y, blk_x, blk_c, nmax, owner);
    /* levels in raster order.  Scanning block j's window finds every block
       that owns a lost pixel in it: an earlier owner is a predecessor of j; a
       later owner has j as a predecessor (j reads the pixel before the owner
       writes it), and is raised above j now -- before its own turn, so every
       level is final when its block's turn comes. */
    int* level = (int*)calloc(nmax + 1, sizeof(int));
    for (int pass = 0; pass < 2 * nb; ++pass) {
        int j = pass / 2, later = pass % 2;
        int c = blk_c[j];
        int B = classes[3 * c], b = classes[3 * c + 1], M = B + 2 * b;
        for (int m = 0; m < M; ++m)
            for (int n = 0; n < M; ++n) {
                int y = blk_y[j] - b + m, x = blk_x[j] - b + n;
                if (y < 0 || y >= H || x < 0 || x >= W) continue;
                int o = owner[(size_t)y * W + x];
                if (o < 0 || o == j) continue;
                if (!later && o < j && level[o] + 1 > level[j]) level[j] = level[o] + 1;
                if (later && o > j && level[j] + 1 > level[o]) level[o] = level[j] + 1;
            }
    }
    int nl = 0;
    for (int j = 0; j < nb; ++j)
        if (level[j] + 1 > nl) nl = level[j] + 1;
    /* blocks grouped by level (counting sort, raster order within a level) */
    int* start = (int*)calloc(nl + 2, sizeof(int));
    int* byl = (int*)malloc(sizeof(int) * (nmax + 1));
    for (int j = 0; j < nb; ++j) start[level[j] + 1]++;
    for (int l = 0; l < nl; ++l) start[l + 1] += start[l];
    int* fill = (int*)malloc(sizeof(int) * (nl + 1));
    for (int l = 0; l <= nl; ++l) fill[l] = start[l];
    for (int j = 0; j < nb; ++j) byl[fill[level[j]]++] = j;

    unsigned char* status = (unsigned char*)malloc((size_t)W * H);
    for (size_t q = 0; q < (size_t)W * H; ++q) {
        out[q] = mask[q] ? 0.0 : img[q];
        status[q] = mask[q] ? ST_LOST : ST_KNOWN;
    }
    int degenerate = 0, threads = 1;
    for (int l = 0; l < nl; ++l) {
#pragma omp parallel for schedule(dynamic, 4) reduction(| : degenerate)
        for (int t = start[l]; t < start[l + 1]; ++t) {
            int bi = byl[t];
            int c = blk_c[bi];
            int K = classes[3 * c + 2];
            int* sel = (int*)malloc(sizeof(int) * (K > 0 ? K : 1));
            double* ar = (double*)malloc(sizeof(double) * (K > 0 ? K : 1));
            double* ai = (double*)malloc(sizeof(double) * (K > 0 ? K : 1));
            double W0 = run_block(bi, blk_y[bi], blk_x[bi], classes + 3 * c, owner, out, status, W, H, rho,
                                  gamma, delta, sel, ar, ai, NULL, NULL);
            degenerate |= (W0 <= 0.0);
            free(sel);
            free(ar);
            free(ai);
        }
    }
#ifdef _OPENMP
    threads = omp_get_max_threads();
#endif
    if (n_levels) *n_levels = nl;
    if (n_threads) *n_threads = threads;
    free(status);
    free(start);
    free(byl);
    free(fill);
    free(level);
    free(owner);
    free(blk_y);
    free(blk_x);
    free(blk_c);
    return degenerate ? -2 : nb;
}
