// Host planner for the tiled stencil executors.
//
// Iteration space of a d-dimensional radius-1 stencil over T steps, after the
// skew (t, i_k) -> (t, j_k = i_k + t) that makes every dependence
// non-negative (paper: Section 4.3.2 Heat-2D skewing; appendix, 1D-Jacobi):
//     0 <= t < T,   1 + t <= j_k <= n_k - 2 + t.
// Dependences in skewed coordinates: (1, delta) with delta_k in {0, 1, 2}.
// Bounding box (Section 4.5): t in [0, T), j_k in [1, n_k - 2 + T - 1].
//
// Tiles (leaves) are b_t x b_1 x ... x b_d boxes aligned at the box's low
// corner.  With the box padded to b * 2^k per dimension the recursive
// halving (Section 4.2) ends exactly on this grid, so single-level tiling and
// the recursive schedules visit the same leaves in different orders; only the
// order differs (Section 1, Section 3.2).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace pcot {

struct StencilGeom {
    int d = 0;                  // spatial dimensions (1..3)
    int64_t n[3] = {0, 0, 0};   // extents incl. boundary, outer..inner (first d used)
    int64_t T = 0;
    int64_t b[4] = {1, 1, 1, 1};  // tile sizes: t, then outer..inner spatial
    int64_t cnt[4] = {1, 1, 1, 1};  // tile-grid counts: t, then spatial
};

// Leaf coordinates: k[0] = time tile, k[1..d] = spatial tiles (outer..inner).
struct Leaf {
    int32_t k[4];
};

StencilGeom make_geom(int d, const int64_t* dims, int64_t T, const int64_t* tile);

// Does the box [lo, lo + size) (skewed coordinates, t first) hold a domain point?
bool box_nonempty(const StencilGeom& g, const int64_t* lo, const int64_t* size);
bool leaf_nonempty(const StencilGeom& g, const int32_t* k);

// Leaves in visiting order for schedule 1..4 (SLT_LEX, SLT_WAVE, COT_SEQ, COT_PAR).
std::vector<Leaf> enumerate_leaves(const StencilGeom& g, int schedule);

// Number of non-empty predecessors (offsets in {0,-1}^(d+1) minus 0).
int count_preds(const StencilGeom& g, const int32_t* k);

// Check that `order` is a topological order of the tile dependence graph and
// covers every non-empty tile exactly once.  Empty string when legal.
std::string check_order(const StencilGeom& g, const std::vector<Leaf>& order);

}  // namespace pcot
