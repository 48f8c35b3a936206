// fse_plan.h -- host planning of processing blocks, dependency keys and
// tiles (internal to libfse).
#pragma once

#include <stdint.h>

#include <vector>

namespace fse {

// entry of the optimised order's heap: a block and its share (fse_plan.cpp)
struct HeapEntry {
    int64_t share;
    int32_t id, cls;
};

struct ClassCfg {
    int B, b, K, M;
};

// Processing blocks of one region (a whole image or one extended tile).
struct RegionPlan {
    int W = 0, H = 0;    // region size
    int fw = 0, fh = 0;  // fine-cell grid (cells of the smallest block edge)
    std::vector<int32_t> owner;  // fw*fh: owning block of the cell's lost pixels, -1 none
    std::vector<int32_t> desc;   // 4 per block: y0, x0, class, 0 (raster order)
    std::vector<int32_t> lbox;   // 4 per block: lost-pixel bounding box y0, x0, y1, x1 (exclusive)
    std::vector<int32_t> key;    // wavefront key per block (a topological order of the dependencies)
    std::vector<int32_t> level;  // longest dependency chain ending at the block (0 = no predecessor)
    int64_t lost_pixels = 0;
};

// Working storage of plan_priority_order, kept between calls.
struct OrderScratch {
    std::vector<int64_t> share;     // per block: usable window weight (exact integer)
    std::vector<HeapEntry> heap;  // max-heap of the blocks not yet processed
    std::vector<int32_t> pos;     // per block, interleaved: heap entry (-1 once processed), dependency level
    std::vector<int32_t> lost_off;  // per block: start of its lost pixels in lost_yx
    std::vector<int32_t> lost_yx;   // lost pixels, (y, x) pairs, grouped by block
    std::vector<int32_t> adj_off;   // per block j: start of its pairs
    std::vector<int32_t> adj_i;     // the blocks whose windows meet j's lost pixels
    std::vector<int64_t> adj_s;     // and what each one's share gains when j is processed
    std::vector<int32_t> perm;      // processing order (raster indices)
    std::vector<int32_t> rank;      // position of every raster block in that order
    std::vector<int64_t> pend;      // the processed block's listed blocks still to come: their gains
    std::vector<int32_t> tmp;       // first block per corner cell, then those blocks' numbers
    std::vector<int64_t> qtab;      // per class: known weights, reconstructed weights, prefix sums
};

// Working storage of plan_region, kept by the caller between calls so that
// repeated planning reuses its memory.
struct PlanScratch {
    std::vector<uint8_t> cells;   // per fine cell: lost count and box (packed)
    std::vector<int8_t> ccls;     // per fine cell: class, -1 none
    std::vector<int32_t> corner;  // per fine cell: block id of a corner cell
    std::vector<uint64_t> bits;   // Bmin mask rows as bit sets
    std::vector<int32_t> cell_level;  // plan_levels: level of each cell's owner
    OrderScratch order;               // plan_priority_order
};

// Block geometry shared by the planner and the kernels: the largest class
// whose aligned square is entirely lost (and inside the region) takes it;
// the smallest class takes every remaining cell holding a lost pixel.
// mask: region view (row pitch in elements).  Returns false on bad classes.
bool plan_region(const uint8_t* mask, int64_t pitch, int W, int H, const std::vector<ClassCfg>& cls,
                 RegionPlan& out, PlanScratch& scratch);

// Dependency level of every block of P (P.level): 1 + the largest level of
// the earlier blocks near it, over a superset of the waits of the block kernel
// (so any order by level still runs every wait on an earlier block).  Sorting
// by level keeps ready blocks ahead of blocks deep in a chain.  cell_level:
// scratch, resized here.
void plan_levels(RegionPlan& P, const std::vector<ClassCfg>& cls, int reach, std::vector<int32_t>& stamp);


// Optimised processing order (Sec. II: large lost areas close from their
// margins towards their centre).  Each step takes the block, among those not
// yet processed, whose support window offers the largest share of usable
// weight -- its sum of R7 weights under the current statuses (rho^dist known,
// delta rho^dist reconstructed, 0 lost or off the region) over that sum for
// a fully known window of its class -- with ties to the raster-earlier block.
// Weights are the integers round(2^30 rho^dist) and round(2^30 delta
// rho^dist), so the shares are exact.  Renumbers the blocks of P in that
// order (desc, lbox, owner), so that a smaller block index still means
// "processed earlier" everywhere, and sets P.level (and P.key = P.level, the
// wavefront schedule's keys): 1 + the largest level of the earlier blocks
// that interact with the block -- exactly the blocks the kernel waits for.
// mask is the region view used to plan P.
// The pair lists and the initial shares are built on up to `threads` host
// threads; the greedy choice itself is sequential.
void plan_priority_order(RegionPlan& P, const uint8_t* mask, int64_t pitch, const std::vector<ClassCfg>& cls,
                         double rho, double delta, OrderScratch& S, int threads);

// Key slope: a block can only interact with blocks whose corner lies at most
// D fine cells to its right in an earlier row, so key = cx + (D + 1) cy
// increases along every dependency.
int key_reach_cells(const std::vector<ClassCfg>& cls);

// Raster-order dependency test of two blocks (i before j): i's lost pixels
// meet j's window, or j's lost pixels meet i's window.
bool blocks_interact(const int32_t* desc_i, const int32_t* lbox_i, const int32_t* desc_j,
                     const int32_t* lbox_j, const std::vector<ClassCfg>& cls);

// Algorithm 1 of the paper (eqs. (1)-(5)): core tiles x, y, w, h.
bool compact_tiling(int W, int H, int N, std::vector<int32_t>& xywh);

// N full-height vertical stripes, widths as eq. (5) with all tiles in one row.
bool vertical_tiling(int W, int H, int N, std::vector<int32_t>& xywh);

}  // namespace fse
