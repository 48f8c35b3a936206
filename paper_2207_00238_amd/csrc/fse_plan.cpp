// fse_plan.cpp -- host planning for libfse.
//
//  * processing blocks of a region from its loss mask, in raster order of
//    their top-left corners, with the owner of every fine cell and the
//    bounding box of every block's lost pixels;
//  * the wavefront key that orders dispatch on the GPU;
//  * the compact tiling of Algorithm 1 (eqs. (1)-(5), Sec. III).
#include "fse_plan.h"

#include <algorithm>

namespace fse {

int key_reach_cells(const std::vector<ClassCfg>& cls) {
    int Bmax = 0, bmax = 0, Bmin = cls.back().B;
    for (const auto& c : cls) {
        Bmax = std::max(Bmax, c.B);
        bmax = std::max(bmax, c.b);
    }
    // corner column distance (in pixels) of interacting blocks is < Bmax + bmax
    return (Bmax + bmax - 1) / Bmin;
}

static inline bool meet(int ay0, int ax0, int ay1, int ax1, int by0, int bx0, int by1, int bx1) {
    return ay0 < by1 && by0 < ay1 && ax0 < bx1 && bx0 < ax1;
}

bool blocks_interact(const int32_t* di, const int32_t* li, const int32_t* dj, const int32_t* lj,
                     const std::vector<ClassCfg>& cls) {
    const ClassCfg& ci = cls[di[2]];
    const ClassCfg& cj = cls[dj[2]];
    const bool a = meet(li[0], li[1], li[2], li[3], dj[0] - cj.b, dj[1] - cj.b, dj[0] + cj.B + cj.b,
                        dj[1] + cj.B + cj.b);
    const bool b = meet(lj[0], lj[1], lj[2], lj[3], di[0] - ci.b, di[1] - ci.b, di[0] + ci.B + ci.b,
                        di[1] + ci.B + ci.b);
    return a || b;
}

bool plan_region(const uint8_t* mask, int64_t pitch, int W, int H, const std::vector<ClassCfg>& cls,
                 RegionPlan& P) {
    const int nc = (int)cls.size();
    if (nc < 1) return false;
    const int Bmin = cls.back().B;
    for (int c = 0; c + 1 < nc; ++c)
        if (cls[c].B % cls[c + 1].B != 0 || cls[c].B <= cls[c + 1].B) return false;
    P.W = W;
    P.H = H;
    P.fw = (W + Bmin - 1) / Bmin;
    P.fh = (H + Bmin - 1) / Bmin;
    const int fw = P.fw, fh = P.fh;
    // per fine cell: any lost pixel, every pixel lost (cell fully inside)
    std::vector<uint8_t> any(fw * (size_t)fh, 0), all(fw * (size_t)fh, 0);
    int64_t lost = 0;
    for (int fy = 0; fy < fh; ++fy)
        for (int fx = 0; fx < fw; ++fx) {
            const int y0 = fy * Bmin, x0 = fx * Bmin;
            const int y1 = std::min(H, y0 + Bmin), x1 = std::min(W, x0 + Bmin);
            int cnt = 0;
            for (int y = y0; y < y1; ++y) {
                const uint8_t* row = mask + (int64_t)y * pitch;
                for (int x = x0; x < x1; ++x) cnt += row[x] != 0;
            }
            lost += cnt;
            any[fy * (size_t)fw + fx] = cnt > 0;
            all[fy * (size_t)fw + fx] = (cnt == Bmin * Bmin);
        }
    P.lost_pixels = lost;
    // class of every fine cell: first (largest) class whose aligned square is
    // entirely lost and inside the region, else the last class if any lost
    std::vector<int8_t> ccls(fw * (size_t)fh, -1);
    for (int fy = 0; fy < fh; ++fy)
        for (int fx = 0; fx < fw; ++fx) {
            int8_t got = -1;
            for (int c = 0; c + 1 < nc && got < 0; ++c) {
                const int f = cls[c].B / Bmin;
                const int cy = fy / f * f, cx = fx / f * f;
                if ((cy + f) * Bmin > H || (cx + f) * Bmin > W) continue;
                bool full = true;
                for (int yy = cy; yy < cy + f && full; ++yy)
                    for (int xx = cx; xx < cx + f; ++xx)
                        if (!all[yy * (size_t)fw + xx]) {
                            full = false;
                            break;
                        }
                if (full) got = (int8_t)c;
            }
            if (got < 0 && any[fy * (size_t)fw + fx]) got = (int8_t)(nc - 1);
            ccls[fy * (size_t)fw + fx] = got;
        }
    // blocks: corner cells in raster order of the fine grid
    P.owner.assign(fw * (size_t)fh, -1);
    P.desc.clear();
    P.lbox.clear();
    P.key.clear();
    const int D = key_reach_cells(cls);
    std::vector<int32_t> corner_id(fw * (size_t)fh, -1);
    for (int fy = 0; fy < fh; ++fy)
        for (int fx = 0; fx < fw; ++fx) {
            const int c = ccls[fy * (size_t)fw + fx];
            if (c < 0) continue;
            const int f = cls[c].B / Bmin;
            if (fy % f || fx % f) continue;
            const int id = (int)(P.desc.size() / 4);
            corner_id[fy * (size_t)fw + fx] = id;
            const int y0 = fy * Bmin, x0 = fx * Bmin;
            P.desc.insert(P.desc.end(), {y0, x0, c, 0});
            // bounding box of the lost pixels
            int ly0 = H, lx0 = W, ly1 = -1, lx1 = -1;
            const int B = cls[c].B;
            for (int y = y0; y < std::min(H, y0 + B); ++y)
                for (int x = x0; x < std::min(W, x0 + B); ++x)
                    if (mask[(int64_t)y * pitch + x]) {
                        ly0 = std::min(ly0, y);
                        lx0 = std::min(lx0, x);
                        ly1 = std::max(ly1, y);
                        lx1 = std::max(lx1, x);
                    }
            P.lbox.insert(P.lbox.end(), {ly0, lx0, ly1 + 1, lx1 + 1});
            P.key.push_back(fx + (D + 1) * fy);
        }
    for (int fy = 0; fy < fh; ++fy)
        for (int fx = 0; fx < fw; ++fx) {
            const int c = ccls[fy * (size_t)fw + fx];
            if (c < 0) continue;
            const int f = cls[c].B / Bmin;
            P.owner[fy * (size_t)fw + fx] = corner_id[(fy / f * f) * (size_t)fw + (fx / f * f)];
        }
    return true;
}

bool compact_tiling(int W, int H, int N, std::vector<int32_t>& xywh) {
    xywh.clear();
    if (W < 1 || H < 1 || N < 1) return false;
    const bool portrait = W < H;
    const int64_t Wl = portrait ? H : W, Hl = portrait ? W : H;
    // eq. (2): n_R = max(1, round(sqrt(N / r))) with r = Wl / Hl (eq. (1)).
    // round(sqrt(q)) = k  iff  (2k - 1)^2 <= 4q < (2k + 1)^2,  4q = 4 N Hl / Wl
    int64_t k = 0;
    while ((2 * k + 1) * (2 * k + 1) * Wl <= 4 * (int64_t)N * Hl) ++k;
    const int64_t nR = std::max<int64_t>(1, k);
    int64_t yT = 0;
    std::vector<int32_t> land;
    for (int64_t i = 1; i <= nR; ++i) {
        // eq. (3): tiles in this row
        const int64_t nC = (i <= N % nR) ? (N + nR - 1) / nR : N / nR;
        // eq. (4): row height; the last row takes what is left
        int64_t hT = (Hl * nC) / N + ((Hl * nC) % N) / nR;
        if (i == nR) hT = Hl - yT;
        // for large N eq. (4) overshoots the image height; rows are clipped at
        // the bottom edge and rows past it stay empty
        hT = std::max<int64_t>(0, std::min<int64_t>(hT, Hl - yT));
        int64_t xT = 0;
        for (int64_t j = 1; j <= nC; ++j) {
            // eq. (5): tile width
            const int64_t wT = (j <= Wl % nC) ? (Wl + nC - 1) / nC : Wl / nC;
            land.insert(land.end(), {(int32_t)xT, (int32_t)yT, (int32_t)wT, (int32_t)hT});
            xT += wT;
        }
        yT += hT;
    }
    if (!portrait) {
        xywh = land;
    } else {
        for (size_t t = 0; t < land.size(); t += 4)
            xywh.insert(xywh.end(), {land[t + 1], land[t], land[t + 3], land[t + 2]});
    }
    return true;
}

}  // namespace fse
