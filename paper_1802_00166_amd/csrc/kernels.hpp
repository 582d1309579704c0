// Host-visible launchers of the HIP kernels (implemented in *.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace pcot {

// Device header words at the start of every workspace.
enum : int {
    HDR_TICKET = 0,  // next ticket of the persistent queue
    HDR_ERROR = 1,   // 0 or a device error code (DEVERR_*)
    HDR_ABORT = 2,   // set once a wait timed out: every block then drains
    HDR_WORDS = 64
};
constexpr unsigned DEVERR_TIMEOUT = 6;
constexpr unsigned DEVERR_INPUT = 7;

hipError_t launch_fill_u32(unsigned* p, size_t n, unsigned v, hipStream_t s);
hipError_t launch_copy_boundary(int dtype, const void* src, void* dst0, void* dst1, int d,
                                const int64_t* n, hipStream_t s);
hipError_t launch_step(int kind, int dtype, const void* src, void* dst, const int64_t* n,
                       hipStream_t s);

// One instance of a tiled stencil problem as the persistent executors see it.
struct TiledProblem {
    const void* in;      // u_0 (read only)
    void* buf0;          // holds u_t for even t >= 2 (and its boundary)
    void* buf1;          // holds u_t for odd t
    int n[3];            // extents, outer..inner (first d used)
    int T;
    int b[4];            // tile sizes: t, outer..inner
    int cnt[4];          // tile-grid counts: t, outer..inner
    unsigned* counters;  // dense over the tile grid
};

// Queue entry: problem index and tile-grid coordinates.
struct QEntry {
    uint16_t k[4];  // time tile, spatial tiles outer..inner
};

struct TiledLaunch {
    const TiledProblem* probs;  // device array of problem descriptors
    const QEntry* queue;        // device array, visiting order
    const uint16_t* qprob;      // device array, problem of each entry (nullptr: all 0)
    int nq;
    unsigned* hdr;              // device header words
    long long limit_ticks;      // watchdog
};

// Writes one problem descriptor to device memory (a kernel, so that it can be
// recorded into a HIP graph).
hipError_t launch_put_problem(TiledProblem* dst, const TiledProblem& v, hipStream_t s);

// Is the tile shape runnable by a tiled executor for (kind, dtype)?
bool tiled_supported(int kind, int dtype, const int* b);
// Launches the persistent tiled executor on `stream`.  `grid_cap` bounds the
// number of blocks (0: fill the device).
hipError_t launch_tiled(int kind, int dtype, const int* b, const TiledLaunch& L, int grid_cap,
                        hipStream_t s);

}  // namespace pcot
