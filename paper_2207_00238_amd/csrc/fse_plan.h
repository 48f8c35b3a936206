// fse_plan.h -- host planning of processing blocks, dependency keys and
// tiles (internal to libfse).
#pragma once

#include <stdint.h>

#include <vector>

namespace fse {

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

// Working storage of plan_region, kept by the caller between calls so that
// repeated planning reuses its memory.
struct PlanScratch {
    std::vector<uint8_t> cells;   // per fine cell: lost count and box (packed)
    std::vector<int8_t> ccls;     // per fine cell: class, -1 none
    std::vector<int32_t> corner;  // per fine cell: block id of a corner cell
    std::vector<uint64_t> bits;   // Bmin mask rows as bit sets
    std::vector<int32_t> cell_level;  // plan_levels: level of each cell's owner
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
