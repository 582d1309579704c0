// Concurrent-start schedules of the 2D stencil: trapezoid tiles from a
// hyperspace cut of every spatial dimension in each time band (the parallel
// space cut of Frigo and Strumpen, as used by Pochoir; the paper's related
// work and its Heat-3D scaling comparison), and the same tiles with the cut
// shifted by half a period in every other band, so that each upright tile
// sits on the inverted tile below it (diamond / hexagonal tiles with
// concurrent start, Bandishti et al.).
//
// Geometry, per spatial dimension, in original (unskewed) coordinates.  A
// band of nt <= bt levels starts at time t0; level l (0 <= l < nt) of a tile
// computes u_{t0+l+1} over [lo + slo*l, hi + shi*l) intersected with the
// interior [1, n-1).  Upright tiles (U) shrink by one point per level on each
// side (slo = +1, shi = -1), inverted tiles (V) grow (slo = -1, shi = +1), and
// a side that lies on the array boundary stays put (slope 0).  U and V tiles
// alternate along the dimension; their level ranges partition the interior at
// every level.  With a footprint of F points (register tile, halo included):
//   U: level-0 width W = F - 2, V: level-0 width g = F - 2 bt, period P = W + g,
// so both kinds hold F - bt - 1 points on average.  In 2D a band has four
// phases (UU, UV, VU, VV: kind in y, kind in x); the tiles of one phase are
// independent, so every phase starts with all its tiles at once.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

namespace pcot {

struct TrapTile {
    int lo[2], hi[2];   // level-0 range per spatial dimension (0 = y, 1 = x)
    int fo[2];          // footprint origin: first array index of the register tile
    int slo[2], shi[2]; // side slopes in {-1, 0, +1}
    int t0, nt;         // first time step of the band, levels of the tile
    int need;           // number of predecessor tiles
    int succ0, nsucc;   // successors: succ[succ0 .. succ0 + nsucc)
    int pad;
};

struct TrapPlanHost {
    std::vector<TrapTile> tiles;  // in queue order (a topological order)
    std::vector<int> succ;
    long long loads = 0, stores = 0;  // algorithmic element transfers of the plan
};

// Schedules 5 (trapezoids) and 6 (shifted by half a period every other band).
// F[0], F[1]: footprints in y and x (F >= 2 bt + 2).  Empty tiles are dropped.
TrapPlanHost build_trap_plan(int ny, int nx, int T, int bt, const int* F, bool shifted);

struct TrapLaunch {
    const TrapTile* tiles;  // device
    const int* succ;        // device
    unsigned* counters;     // device, one per tile, zeroed before the launch
    unsigned* hdr;          // device header words (ticket, error, abort)
    const void* in;         // u_0
    void* buf0;             // u_t for even t >= 2
    void* buf1;             // u_t for odd t
    int ntiles;
    int ny, nx;
    long long limit_ticks;
};

bool trap2d_supported(int dtype, int bt, int fy, int fx);
hipError_t launch_trap2d(int dtype, int bt, int fy, int fx, const TrapLaunch& L, hipStream_t s);

}  // namespace pcot
