// fse_plan.cpp -- host planning for libfse.
//
//  * processing blocks of a region from its loss mask, in raster order of
//    their top-left corners, with the owner of every fine cell and the
//    bounding box of every block's lost pixels;
//  * the wavefront key that orders dispatch on the GPU;
//  * the compact tiling of Algorithm 1 (eqs. (1)-(5), Sec. III).
#include "fse_plan.h"

#include <algorithm>
#if defined(__SSE2__)
#include <emmintrin.h>
#endif

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

// Lost-pixel bit set of one mask row: bit x%64 of word x/64 is set when
// pixel x is lost.  Sixteen bytes at a time where SSE2 is there.
static void row_bits(const uint8_t* row, int W, uint64_t* out) {
    const int nw = (W + 63) / 64;
    for (int w = 0; w < nw; ++w) out[w] = 0;
    int x = 0;
#if defined(__SSE2__)
    const __m128i z = _mm_setzero_si128();
    for (; x + 16 <= W; x += 16) {
        const __m128i v = _mm_loadu_si128(reinterpret_cast<const __m128i*>(row + x));
        const uint32_t zero = (uint32_t)_mm_movemask_epi8(_mm_cmpeq_epi8(v, z));
        out[x >> 6] |= (uint64_t)(~zero & 0xFFFFu) << (x & 63);
    }
#endif
    for (; x < W; ++x) out[x >> 6] |= (uint64_t)(row[x] != 0) << (x & 63);
}

namespace {

struct CellStat {
    uint16_t cnt;            // lost pixels in the cell
    uint8_t y0, y1, x0, x1;  // their bounding box, cell-relative
};

// popcount of one byte without a CPU popcount instruction
struct Popc8 {
    uint8_t v[256];
    constexpr Popc8() : v() {
        for (int i = 0; i < 256; ++i) v[i] = (uint8_t)((i & 1) + ((i >> 1) & 1) + ((i >> 2) & 1) + ((i >> 3) & 1) +
                                                       ((i >> 4) & 1) + ((i >> 5) & 1) + ((i >> 6) & 1) + (i >> 7));
    }
};
constexpr Popc8 kPopc8;

// Cell statistics of one row of fine cells from its BM mask rows (ny <= BM
// rows at the bottom edge), given as bit sets of nw64 words each.  BM divides
// 64, so a cell never straddles two words.  Cells without lost pixels are
// skipped word by word.
template <int BM>
int64_t cell_row(const uint64_t* rb, int nw64, int ny, int fw, CellStat* crow) {
    constexpr uint64_t CM = BM == 64 ? ~0ull : ((1ull << BM) - 1);
    constexpr int PER = 64 / BM;  // cells per word
    int64_t lost = 0;
    for (int w = 0; w < nw64; ++w) {
        uint64_t orw = 0;
        for (int r = 0; r < ny; ++r) orw |= rb[(size_t)r * nw64 + w];
        const int fx0 = w * PER, fx1 = std::min(fw, fx0 + PER);
        for (int fx = fx0; fx < fx1; ++fx) crow[fx] = CellStat{0, 255, 0, 255, 0};
        while (orw) {
            const int k = __builtin_ctzll(orw) / BM;  // cell within the word
            orw &= ~(CM << (k * BM));
            const int fx = fx0 + k;
            if (fx >= fw) break;
            uint32_t any = 0;
            int n = 0, y0 = 255, y1 = 0;
            for (int r = 0; r < ny; ++r) {
                const uint32_t bits = (uint32_t)((rb[(size_t)r * nw64 + w] >> (k * BM)) & CM);
                any |= bits;
                n += kPopc8.v[bits & 255] + kPopc8.v[(bits >> 8) & 255];
                y0 = (bits && y0 == 255) ? r : y0;
                y1 = bits ? r + 1 : y1;
            }
            crow[fx] = CellStat{(uint16_t)n, (uint8_t)y0, (uint8_t)y1, (uint8_t)__builtin_ctz(any),
                                (uint8_t)(32 - __builtin_clz(any))};
            lost += n;
        }
    }
    return lost;
}

}  // namespace

bool plan_region(const uint8_t* mask, int64_t pitch, int W, int H, const std::vector<ClassCfg>& cls,
                 RegionPlan& P, PlanScratch& S) {
    const int nc = (int)cls.size();
    if (nc < 1) return false;
    const int Bmin = cls.back().B;
    if (Bmin != 1 && Bmin != 2 && Bmin != 4 && Bmin != 8 && Bmin != 16) return false;
    for (int c = 0; c + 1 < nc; ++c)
        if (cls[c].B % cls[c + 1].B != 0 || cls[c].B <= cls[c + 1].B) return false;
    P.W = W;
    P.H = H;
    P.fw = (W + Bmin - 1) / Bmin;
    P.fh = (H + Bmin - 1) / Bmin;
    const int fw = P.fw, fh = P.fh;
    const size_t ncell = fw * (size_t)fh;
    // pass 1, row-major over the mask: per fine cell the number of lost
    // pixels and their bounding box
    S.cells.resize(ncell * sizeof(CellStat));
    CellStat* cs = reinterpret_cast<CellStat*>(S.cells.data());
    const int nw64 = (W + 63) / 64;
    S.bits.resize((size_t)nw64 * Bmin);
    uint64_t* rb = S.bits.data();
    int64_t lost = 0;
    for (int fy = 0; fy < fh; ++fy) {
        const int ny = std::min(Bmin, H - fy * Bmin);
        for (int r = 0; r < ny; ++r) row_bits(mask + (int64_t)(fy * Bmin + r) * pitch, W, rb + (size_t)r * nw64);
        CellStat* crow = cs + fy * (size_t)fw;
        switch (Bmin) {
            case 1: lost += cell_row<1>(rb, nw64, ny, fw, crow); break;
            case 2: lost += cell_row<2>(rb, nw64, ny, fw, crow); break;
            case 4: lost += cell_row<4>(rb, nw64, ny, fw, crow); break;
            case 8: lost += cell_row<8>(rb, nw64, ny, fw, crow); break;
            default: lost += cell_row<16>(rb, nw64, ny, fw, crow); break;
        }
    }
    P.lost_pixels = lost;
    // pass 2: class of every fine cell -- the first (largest) class whose
    // aligned square is entirely lost and inside the region, else the last
    // class if any pixel is lost -- and the number of blocks (corner cells)
    const int full_cnt = Bmin * Bmin;
    S.ccls.resize(ncell);
    int8_t* ccls = S.ccls.data();
    size_t nblk = 0;
    for (int fy = 0; fy < fh; ++fy)
        for (int fx = 0; fx < fw; ++fx) {
            const size_t q = fy * (size_t)fw + fx;
            int8_t got = -1;
            if (cs[q].cnt) {
                for (int c = 0; c + 1 < nc && got < 0; ++c) {
                    const int f = cls[c].B / Bmin;
                    const int cy = fy / f * f, cx = fx / f * f;
                    if ((cy + f) * Bmin > H || (cx + f) * Bmin > W) continue;
                    bool full = true;
                    for (int yy = cy; yy < cy + f && full; ++yy)
                        for (int xx = cx; xx < cx + f; ++xx)
                            if (cs[yy * (size_t)fw + xx].cnt != full_cnt) {
                                full = false;
                                break;
                            }
                    if (full) got = (int8_t)c;
                }
                if (got < 0) got = (int8_t)(nc - 1);
                const int f = cls[got].B / Bmin;
                nblk += (fy % f == 0 && fx % f == 0);
            }
            ccls[q] = got;
        }
    // pass 3: blocks at corner cells in raster order of the fine grid, and
    // the owner of every cell (a square's corner comes first in raster order)
    P.owner.resize(ncell);
    P.desc.resize(4 * nblk);
    P.lbox.resize(4 * nblk);
    P.key.resize(nblk);
    const int D = key_reach_cells(cls);
    S.corner.resize(ncell);
    int32_t* corner_id = S.corner.data();
    int32_t* owner = P.owner.data();
    size_t id = 0;
    for (int fy = 0; fy < fh; ++fy)
        for (int fx = 0; fx < fw; ++fx) {
            const size_t q = fy * (size_t)fw + fx;
            const int c = ccls[q];
            if (c < 0) {
                owner[q] = -1;
                continue;
            }
            const int f = cls[c].B / Bmin;
            if (fy % f || fx % f) {
                owner[q] = corner_id[(fy / f * f) * (size_t)fw + (fx / f * f)];
                continue;
            }
            corner_id[q] = (int32_t)id;
            owner[q] = (int32_t)id;
            const int y0 = fy * Bmin, x0 = fx * Bmin;
            int32_t* dd = &P.desc[4 * id];
            dd[0] = y0;
            dd[1] = x0;
            dd[2] = c;
            dd[3] = 0;
            // bounding box of the lost pixels: a larger class owns a fully lost
            // square; the smallest class owns one cell
            int32_t* lb = &P.lbox[4 * id];
            if (c + 1 < nc) {
                lb[0] = y0;
                lb[1] = x0;
                lb[2] = y0 + cls[c].B;
                lb[3] = x0 + cls[c].B;
            } else {
                lb[0] = y0 + cs[q].y0;
                lb[1] = x0 + cs[q].x0;
                lb[2] = y0 + cs[q].y1;
                lb[3] = x0 + cs[q].x1;
            }
            P.key[id] = fx + (D + 1) * fy;
            ++id;
        }
    return true;
}

void plan_levels(RegionPlan& P, const std::vector<ClassCfg>& cls, int reach, std::vector<int32_t>& cell_level) {
    // Levels over a superset of the kernel's waits: every earlier block owning
    // a fine cell in the rows of the kernel's scan up to the block's own corner
    // row (every earlier block the kernel's scan finds owns such a cell).  A
    // superset of the edges still orders every real wait, and needs no box
    // tests: a running maximum over the cells, each cell holding the level of
    // its owner once that block has been assigned one (-1 before).
    const size_t nb = P.key.size();
    P.level.resize(nb);
    const int Bmin = cls.back().B;
    const int fw = P.fw;
    cell_level.assign(P.owner.size(), -1);
    for (size_t j = 0; j < nb; ++j) {
        const int32_t* dj = &P.desc[4 * j];
        const int Bj = cls[dj[2]].B;
        const int ry0 = dj[0] - reach, rx0 = dj[1] - reach;
        const int rx1 = dj[1] + Bj + reach;
        const int fy0 = std::max(0, ry0 >= 0 ? ry0 / Bmin : 0), fx0 = std::max(0, rx0 >= 0 ? rx0 / Bmin : 0);
        const int fx1 = std::min(fw - 1, (rx1 - 1) / Bmin);
        const int fyj = dj[0] / Bmin, fxj = dj[1] / Bmin;
        int m = -1;
        for (int fy = fy0; fy <= fyj; ++fy) {
            const int32_t* row = &cell_level[(size_t)fy * fw];
            for (int fx = fx0; fx <= fx1; ++fx) m = std::max(m, row[fx]);
        }
        const int lv = m + 1;
        P.level[j] = lv;
        const int f = Bj / Bmin;
        for (int fy = fyj; fy < std::min(P.fh, fyj + f); ++fy)
            for (int fx = fxj; fx < std::min(fw, fxj + f); ++fx) cell_level[(size_t)fy * fw + fx] = lv;
    }
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

bool vertical_tiling(int W, int H, int N, std::vector<int32_t>& xywh) {
    xywh.clear();
    if (W < 1 || H < 1 || N < 1) return false;
    int64_t xT = 0;
    for (int64_t j = 1; j <= N; ++j) {
        const int64_t wT = (j <= W % N) ? (W + N - 1) / N : W / N;
        xywh.insert(xywh.end(), {(int32_t)xT, 0, (int32_t)wT, (int32_t)H});
        xT += wT;
    }
    return true;
}

}  // namespace fse
