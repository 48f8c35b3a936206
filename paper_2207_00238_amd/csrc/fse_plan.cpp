// fse_plan.cpp -- host planning for libfse.
//
//  * processing blocks of a region from its loss mask, in raster order of
//    their top-left corners, with the owner of every fine cell and the
//    bounding box of every block's lost pixels;
//  * the wavefront key that orders dispatch on the GPU;
//  * the compact tiling of Algorithm 1 (eqs. (1)-(5), Sec. III).
#include "fse_plan.h"

#include <algorithm>
#include <cmath>
#include <thread>
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

// ---------------------------------------------------------------------------
// optimised processing order
// ---------------------------------------------------------------------------
namespace {

typedef unsigned __int128 u128;
constexpr int kMaxPlanClasses = 8;

// fn(t, i0, i1) for nt contiguous chunks [i0, i1) of [0, n), chunk t on a
// thread of its own (the calling thread takes the last)
template <class F>
void run_chunks(int n, int nt, F&& fn) {
    std::vector<std::thread> th;
    th.reserve(nt > 1 ? nt - 1 : 0);
    for (int t = 0; t + 1 < nt; ++t)
        th.emplace_back([&, t] { fn(t, (int)((int64_t)n * t / nt), (int)((int64_t)n * (t + 1) / nt)); });
    fn(nt - 1, (int)((int64_t)n * (nt - 1) / nt), n);
    for (auto& x : th) x.join();
}

// Indexed binary max-heap of blocks: a block ranks higher when its share of
// usable weight is larger (share / full of its class, compared exactly by
// cross-multiplication), then when its raster index is smaller.  Each entry
// carries its block's share, so comparisons read the heap array only.
struct ShareHeap {
    const int64_t* full;  // per class
    HeapEntry* heap;
    int32_t* pos;         // entry of every block (stride 2), -1 once popped
    int n = 0;
    bool one_full = false;  // every class has the same full-window weight: compare shares directly
    bool above(const HeapEntry& a, const HeapEntry& b) const {
        if (one_full) return a.share > b.share || (a.share == b.share && a.id < b.id);
        const u128 l = (u128)(uint64_t)a.share * (uint64_t)full[b.cls];
        const u128 r = (u128)(uint64_t)b.share * (uint64_t)full[a.cls];
        return l > r || (l == r && a.id < b.id);
    }
    void place(int k, const HeapEntry& e) {
        heap[k] = e;
        pos[2 * e.id] = k;
    }
    void up(int k) {
        const HeapEntry e = heap[k];
        while (k > 0) {
            const int parent = (k - 1) >> 1;
            if (!above(e, heap[parent])) break;
            place(k, heap[parent]);
            k = parent;
        }
        place(k, e);
    }
    void down(int k) {
        const HeapEntry e = heap[k];
        for (;;) {
            int c = 2 * k + 1;
            if (c >= n) break;
            if (c + 1 < n && above(heap[c + 1], heap[c])) ++c;
            if (!above(heap[c], e)) break;
            place(k, heap[c]);
            k = c;
        }
        place(k, e);
    }
    // block i's share grows by d
    void raise(int i, int64_t d) {
        heap[pos[2 * i]].share += d;
        up(pos[2 * i]);
    }
    int pop() {
        const int top = heap[0].id;
        pos[2 * top] = -1;
        if (--n > 0) {
            place(0, heap[n]);
            down(0);
        }
        return top;
    }
};

}  // namespace

void plan_priority_order(RegionPlan& P, const uint8_t* mask, int64_t pitch, const std::vector<ClassCfg>& cls,
                         double rho, double delta, OrderScratch& S, int threads) {
    const int n = (int)(P.desc.size() / 4);
    const int nc = (int)cls.size();
    if (n <= 1 || nc > kMaxPlanClasses) {
        P.level.assign(n, 0);
        P.key = P.level;
        return;
    }
    const int Bmin = cls.back().B;
    // integer weights per class: known and reconstructed, each with its 2-D
    // prefix sum (sums over rectangles of the window in O(1))
    std::vector<size_t> t_known(nc), t_rec(nc), t_pk(nc), t_pr(nc);
    std::vector<int64_t> full(nc);
    size_t tot = 0;
    for (int c = 0; c < nc; ++c) {
        const size_t MM = (size_t)cls[c].M * cls[c].M, M1 = (size_t)(cls[c].M + 1) * (cls[c].M + 1);
        t_known[c] = tot;
        t_rec[c] = tot + MM;
        t_pk[c] = tot + 2 * MM;
        t_pr[c] = tot + 2 * MM + M1;
        tot += 2 * MM + 2 * M1;
    }
    S.qtab.assign(tot, 0);
    for (int c = 0; c < nc; ++c) {
        const int M = cls[c].M;
        int64_t* qk = &S.qtab[t_known[c]];
        int64_t* qr = &S.qtab[t_rec[c]];
        const double mid = 0.5 * (M - 1);
        for (int m = 0; m < M; ++m)
            for (int k = 0; k < M; ++k) {
                const double dy = m - mid, dx = k - mid;
                const double w = std::pow(rho, std::sqrt(dy * dy + dx * dx));
                qk[m * M + k] = std::llround(std::ldexp(w, 30));
                qr[m * M + k] = std::llround(std::ldexp(delta * w, 30));
            }
        for (int t = 0; t < 2; ++t) {
            const int64_t* q = t ? qr : qk;
            int64_t* pre = &S.qtab[t ? t_pr[c] : t_pk[c]];
            for (int m = 0; m < M; ++m)
                for (int k = 0; k < M; ++k)
                    pre[(m + 1) * (M + 1) + k + 1] =
                        q[m * M + k] + pre[m * (M + 1) + k + 1] + pre[(m + 1) * (M + 1) + k] - pre[m * (M + 1) + k];
        }
        full[c] = S.qtab[t_pk[c] + (size_t)M * (M + 1) + M];
    }
    // sum of a prefix-summed table over rows [m0, m1) and columns [k0, k1)
    auto rect = [](const int64_t* pre, int M, int m0, int m1, int k0, int k1) -> int64_t {
        if (m1 <= m0 || k1 <= k0) return 0;
        return pre[m1 * (M + 1) + k1] - pre[m0 * (M + 1) + k1] - pre[m1 * (M + 1) + k0] + pre[m0 * (M + 1) + k0];
    };
    const int nth = std::max(1, std::min(threads, n / 256 + 1));
    // lost pixels of every block, grouped by block: counted, then filled, by
    // chunks of blocks on threads of their own
    auto lost_scan = [&](int j, auto&& fn) {
        const int32_t* lb = &P.lbox[4 * (size_t)j];
        for (int y = lb[0]; y < lb[2]; ++y)
            for (int x = lb[1]; x < lb[3]; ++x)
                if (mask[(int64_t)y * pitch + x] && P.owner[(size_t)(y / Bmin) * P.fw + x / Bmin] == j) fn(y, x);
    };
    S.lost_off.assign(n + 1, 0);
    run_chunks(n, nth, [&](int, int j0, int j1) {
        for (int j = j0; j < j1; ++j) {
            int cnt = 0;
            lost_scan(j, [&](int, int) { ++cnt; });
            S.lost_off[j + 1] = cnt;
        }
    });
    for (int j = 0; j < n; ++j) S.lost_off[j + 1] += S.lost_off[j];
    S.lost_yx.resize(2 * (size_t)S.lost_off[n]);
    run_chunks(n, nth, [&](int, int j0, int j1) {
        for (int j = j0; j < j1; ++j) {
            int32_t* out = S.lost_yx.data() + 2 * (size_t)S.lost_off[j];
            lost_scan(j, [&](int y, int x) {
                *out++ = y;
                *out++ = x;
            });
        }
    });
    // every block i whose window meets the lost pixels of block j:
    // fn(i, sum over those pixels of table t of i's class, at their window
    // positions); table 0 = known weights, 1 = reconstructed weights
    int Rmax = 0;
    for (auto& c : cls) Rmax = std::max(Rmax, c.B + c.b);
    // raw views of the tables the scans read
    const int32_t* desc = P.desc.data();
    const int32_t* lbox = P.lbox.data();
    const int32_t* loff = S.lost_off.data();
    const int32_t* lyx = S.lost_yx.data();
    const int64_t* qtab = S.qtab.data();
    const int fh = P.fh;
    int cb[kMaxPlanClasses], cM[kMaxPlanClasses];
    size_t tk[kMaxPlanClasses], tr[kMaxPlanClasses], pk[kMaxPlanClasses], pr[kMaxPlanClasses];
    for (int c = 0; c < nc; ++c) {
        cb[c] = cls[c].b;
        cM[c] = cls[c].M;
        tk[c] = t_known[c];
        tr[c] = t_rec[c];
        pk[c] = t_pk[c];
        pr[c] = t_pr[c];
    }
    // blocks by corner cell: the blocks are in raster order of their corner
    // cells, so first[fy][fx] -- the first block whose corner is in row fy at
    // column >= fx (fx = 0 .. fw) -- bounds every row's run of blocks
    const int fw1 = P.fw + 1;
    S.tmp.resize((size_t)fw1 * fh + 1);
    int32_t* first = S.tmp.data();
    {
        int i = 0;
        for (int fy = 0; fy < fh; ++fy)
            for (int fx = 0; fx <= P.fw; ++fx) {
                while (i < n && (desc[4 * i] / Bmin < fy || (desc[4 * i] / Bmin == fy && desc[4 * i + 1] / Bmin < fx)))
                    ++i;
                first[(size_t)fy * fw1 + fx] = i;
            }
        first[(size_t)fw1 * fh] = n;
    }
    int bmax = 0;
    for (auto& c : cls) bmax = std::max(bmax, c.b);
    // every block i whose window meets the lost box of block j: its corner
    // lies within rows (lb0 - B_i - b_i, lb2 + b_i) and the same columns;
    // fn(i, sum of table t of i's class over j's lost pixels in i's window)
    // with t = 0 the known weights, 1 the reconstructed ones
    auto pixel_sum = [&](int j, int c, int wy, int wx, int table) -> int64_t {
        const int32_t* lb = &lbox[4 * j];
        const int M = cM[c];
        if ((int64_t)(loff[j + 1] - loff[j]) == (int64_t)(lb[2] - lb[0]) * (lb[3] - lb[1]))
            // every pixel of the box is lost: one rectangle of the table
            return rect(qtab + (table ? pr[c] : pk[c]), M, std::max(0, lb[0] - wy), std::min(M, lb[2] - wy),
                        std::max(0, lb[1] - wx), std::min(M, lb[3] - wx));
        const int64_t* q = qtab + (table ? tr[c] : tk[c]);
        int64_t sum = 0;
        for (int k = loff[j]; k < loff[j + 1]; ++k) {
            const int m = lyx[2 * k] - wy, x = lyx[2 * k + 1] - wx;
            if (m >= 0 && m < M && x >= 0 && x < M) sum += q[m * M + x];
        }
        return sum;
    };
    auto for_windows_meeting = [&](int j, auto&& fn) {
        const int32_t* lb = &lbox[4 * j];
        const int fy0 = std::max(0, (lb[0] - Rmax + 1) / Bmin), fy1 = std::min(fh - 1, (lb[2] + bmax - 1) / Bmin);
        const int fx0 = std::max(0, (lb[1] - Rmax + 1) / Bmin), fx1 = std::min(P.fw - 1, (lb[3] + bmax - 1) / Bmin);
        for (int fy = fy0; fy <= fy1; ++fy) {
            const int i1 = first[(size_t)fy * fw1 + fx1 + 1];
            for (int i = first[(size_t)fy * fw1 + fx0]; i < i1; ++i) {
                const int32_t* di = &desc[4 * i];
                const int c = di[2], M = cM[c];
                const int wy = di[0] - cb[c], wx = di[1] - cb[c];
                if (meet(lb[0], lb[1], lb[2], lb[3], wy, wx, wy + M, wx + M)) fn(i, c, wy, wx);
            }
        }
    };
    // the pairs, by j: every i whose window meets j's lost box, with the sum
    // of i's reconstructed weights over j's lost pixels (what i's share gains
    // when j is processed).  Counted, then filled in place, by chunks of
    // blocks on threads of their own.
    S.adj_off.assign(n + 1, 0);
    run_chunks(n, nth, [&](int, int j0, int j1) {
        for (int j = j0; j < j1; ++j) {
            int cnt = 0;
            for_windows_meeting(j, [&](int, int, int, int) { ++cnt; });
            S.adj_off[j + 1] = cnt;
        }
    });
    for (int j = 0; j < n; ++j) S.adj_off[j + 1] += S.adj_off[j];
    S.adj_i.resize(S.adj_off[n]);
    S.adj_s.resize(S.adj_off[n]);
    run_chunks(n, nth, [&](int, int j0, int j1) {
        for (int j = j0; j < j1; ++j) {
            int e = S.adj_off[j];
            for_windows_meeting(j, [&](int i, int c, int wy, int wx) {
                S.adj_i[e] = i;
                S.adj_s[e] = pixel_sum(j, c, wy, wx, 1);
                ++e;
            });
        }
    });
    // initial shares, per block i on the threads: known weights of its window
    // inside the region, minus those of the lost pixels in it (the lost boxes
    // that meet the window: corners within rows (wy - Bmax, wy + M))
    int Bmax = 0;
    for (auto& c : cls) Bmax = std::max(Bmax, c.B);
    S.share.resize(n);
    run_chunks(n, nth, [&](int, int i0, int i1) {
        for (int i = i0; i < i1; ++i) {
            const int32_t* di = &desc[4 * i];
            const int c = di[2], M = cM[c];
            const int wy = di[0] - cb[c], wx = di[1] - cb[c];
            int64_t sh = rect(qtab + pk[c], M, std::max(0, -wy), std::min(M, P.H - wy), std::max(0, -wx),
                              std::min(M, P.W - wx));
            const int fy0 = std::max(0, (wy - Bmax + 1) / Bmin), fy1 = std::min(fh - 1, (wy + M - 1) / Bmin);
            const int fx0 = std::max(0, (wx - Bmax + 1) / Bmin), fx1 = std::min(P.fw - 1, (wx + M - 1) / Bmin);
            for (int fy = fy0; fy <= fy1; ++fy) {
                const int j1 = first[(size_t)fy * fw1 + fx1 + 1];
                for (int j = first[(size_t)fy * fw1 + fx0]; j < j1; ++j) {
                    const int32_t* lb = &lbox[4 * j];
                    if (meet(lb[0], lb[1], lb[2], lb[3], wy, wx, wy + M, wx + M)) sh -= pixel_sum(j, c, wy, wx, 0);
                }
            }
            S.share[i] = sh;
        }
    });
    // greedy: the best remaining block; its lost pixels turn reconstructed.
    // The dependency levels of that order come along, over exactly the waits
    // of the block kernel: two blocks interact when either one's lost box
    // meets the other's window -- each such pair is some (j, i in j's list).
    // When j is processed it takes its level from the listed blocks processed
    // before it (and from the raises it received from earlier blocks whose
    // lists hold it), then raises the listed blocks still to come.
    S.heap.resize(n);
    S.pos.resize(2 * (size_t)n);  // per block: heap entry (-1 once processed), level
    ShareHeap hp{full.data(), S.heap.data(), S.pos.data(), n};
    hp.one_full = std::all_of(full.begin(), full.end(), [&](int64_t f) { return f == full[0]; });
    for (int i = 0; i < n; ++i) {
        hp.place(i, HeapEntry{S.share[i], i, desc[4 * i + 2]});
        S.pos[2 * (size_t)i + 1] = 0;
    }
    for (int k = n / 2 - 1; k >= 0; --k) hp.down(k);
    S.perm.resize(n);
    const int32_t* aoff = S.adj_off.data();
    const int32_t* ai = S.adj_i.data();
    const int64_t* as = S.adj_s.data();
    int32_t* pl = S.pos.data();
    int deg = 0;
    for (int j = 0; j < n; ++j) deg = std::max(deg, aoff[j + 1] - aoff[j]);
    S.tmp.resize(deg);
    S.pend.resize(deg);
    int32_t* pend_i = S.tmp.data();
    int64_t* pend_s = S.pend.data();
    for (int k = 0; k < n; ++k) {
        const int j = hp.pop();  // its heap entry is -1 from here on
        S.perm[k] = j;
        // one pass over j's list: the level from the blocks processed before
        // it, and the blocks still to come
        int lv = pl[2 * j + 1], np = 0;
        for (int e = aoff[j]; e < aoff[j + 1]; ++e) {
            const int i = ai[e];  // (j's own window meets its lost box: j is in its list)
            if (pl[2 * i] < 0) {
                if (i != j && pl[2 * i + 1] + 1 > lv) lv = pl[2 * i + 1] + 1;
            } else {
                pend_i[np] = i;
                pend_s[np++] = as[e];
            }
        }
        pl[2 * j + 1] = lv;
        for (int u = 0; u < np; ++u) {
            const int i = pend_i[u];
            if (pl[2 * i + 1] < lv + 1) pl[2 * i + 1] = lv + 1;
            if (pend_s[u] != 0) hp.raise(i, pend_s[u]);
        }
    }
    S.rank.resize(n);
    for (int k = 0; k < n; ++k) S.rank[S.perm[k]] = k;
    // renumber: block k of the plan is the k-th processed
    std::vector<int32_t> d2(4 * (size_t)n), l2(4 * (size_t)n);
    P.level.resize(n);
    const int no = (int)P.owner.size();
    run_chunks(std::max(n, no), nth, [&](int, int k0, int k1) {
        for (int c = k0; c < std::min(k1, no); ++c)
            if (P.owner[c] >= 0) P.owner[c] = S.rank[P.owner[c]];
        for (int k = k0; k < std::min(k1, n); ++k) {
            const size_t src = 4 * (size_t)S.perm[k];
            for (int q = 0; q < 4; ++q) {
                d2[4 * (size_t)k + q] = P.desc[src + q];
                l2[4 * (size_t)k + q] = P.lbox[src + q];
            }
            P.level[k] = S.pos[2 * (size_t)S.perm[k] + 1];
        }
    });
    P.desc.swap(d2);
    P.lbox.swap(l2);
    P.key = P.level;
}

// Tiles of one row holding n tiles of a length L: eq. (5) gives the first
// L mod n tiles the width ceil(L / n) and the rest floor(L / n), so tile j
// (0-based) starts at j floor(L / n) + min(j, L mod n).
static inline int64_t split_start(int64_t L, int64_t n, int64_t j) { return j * (L / n) + std::min(j, L % n); }

bool compact_tiling(int W, int H, int N, std::vector<int32_t>& xywh) {
    xywh.clear();
    if (W < 1 || H < 1 || N < 1) return false;
    // portrait images are tiled as their transpose (landscape is assumed)
    const bool portrait = W < H;
    const int64_t Wl = portrait ? H : W, Hl = portrait ? W : H;
    // eqs. (1)-(2): rows nR = max(1, round(sqrt(N / r))), r = Wl / Hl, with
    // round(sqrt(q)) = k  iff  (2k - 1)^2 <= 4q < (2k + 1)^2 and 4q = 4 N Hl / Wl
    int64_t k = 0;
    while ((2 * k + 1) * (2 * k + 1) * Wl <= 4 * (int64_t)N * Hl) ++k;
    const int64_t nR = std::max<int64_t>(1, k);
    // eq. (3): the first N mod nR rows hold ceil(N / nR) tiles, the others
    // floor(N / nR); eq. (4) then gives one height per kind of row
    const int64_t n_hi = (N + nR - 1) / nR, n_lo = N / nR, rows_hi = N % nR;
    auto height = [&](int64_t nC) { return (Hl * nC) / N + ((Hl * nC) % N) / nR; };
    const int64_t h_hi = height(n_hi), h_lo = height(n_lo);
    // row i (0-based) starts below i rows: min(i, rows_hi) of height h_hi and
    // the rest of height h_lo; the last row reaches the bottom edge.  For
    // large N eq. (4) can pass the bottom edge: rows are clipped there, and
    // rows below it are empty.
    auto row_top = [&](int64_t i) { return std::min(Hl, std::min(i, rows_hi) * h_hi + std::max<int64_t>(0, i - rows_hi) * h_lo); };
    for (int64_t i = 0; i < nR; ++i) {
        const int64_t y0 = row_top(i), y1 = (i + 1 == nR) ? Hl : row_top(i + 1);
        const int64_t nC = i < rows_hi ? n_hi : n_lo;
        for (int64_t j = 0; j < nC; ++j) {
            const int64_t x0 = split_start(Wl, nC, j), x1 = split_start(Wl, nC, j + 1);
            if (!portrait)
                xywh.insert(xywh.end(), {(int32_t)x0, (int32_t)y0, (int32_t)(x1 - x0), (int32_t)(y1 - y0)});
            else
                xywh.insert(xywh.end(), {(int32_t)y0, (int32_t)x0, (int32_t)(y1 - y0), (int32_t)(x1 - x0)});
        }
    }
    return true;
}

bool vertical_tiling(int W, int H, int N, std::vector<int32_t>& xywh) {
    xywh.clear();
    if (W < 1 || H < 1 || N < 1) return false;
    for (int64_t j = 0; j < N; ++j) {
        const int64_t x0 = split_start(W, N, j), x1 = split_start(W, N, j + 1);
        xywh.insert(xywh.end(), {(int32_t)x0, 0, (int32_t)(x1 - x0), (int32_t)H});
    }
    return true;
}

}  // namespace fse
