// Host-visible launchers of the HIP kernels (implemented in *.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <exception>
#include <new>

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
hipError_t launch_fill_chain(long long* p, int n, long long pmax, hipStream_t s);
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
hipError_t launch_put_problems(TiledProblem* dst, const TiledProblem* v, int n, hipStream_t s);
// Boundary of every problem's u_0 into both of its buffers (one launch).
hipError_t launch_copy_boundary_batched(int dtype, const TiledProblem* probs, int nprob, int d, hipStream_t s);

// Error norms (binary64): `scratch` holds norms_scratch_bytes(); the four
// results land at the end of it.
size_t norms_scratch_bytes();
// Same two passes with the final four values written to `result` (device).
hipError_t launch_norms_to(int dtype, int d, const int64_t* n, const void* x, const double* r, double* scratch,
                           double* result, hipStream_t s);
// Device address of the library's static partials array on the current
// device (looked up once per device); its size in bytes.
hipError_t norms_static_scratch(double** out);
size_t norms_static_scratch_bytes();
hipError_t launch_norms(int dtype, int d, const int64_t* n, const void* x, const double* r, double* scratch,
                        hipStream_t s);

// Sets the thread's last-error message and returns `code` (api.cpp).
int32_t fail(int32_t code, const char* fmt, ...);

// No C++ exception may cross the C ABI: every extern "C" entry point wraps
// its body in PCOT_TRY ... PCOT_CATCH(value returned on failure), which turns
// a host allocation failure (std::bad_alloc from a plan or sweep container)
// or any other exception into PCOT_ERR_HOST with a message.
#define PCOT_TRY try {
#define PCOT_CATCH(onerr)                                                                 \
    }                                                                                     \
    catch (const std::bad_alloc&) {                                                       \
        pcot::fail(-8, "host memory allocation failed");                                  \
        return onerr;                                                                     \
    }                                                                                     \
    catch (const std::exception& e_) {                                                    \
        pcot::fail(-8, "host exception: %s", e_.what());                                  \
        return onerr;                                                                     \
    }                                                                                     \
    catch (...) {                                                                         \
        pcot::fail(-8, "unknown host exception");                                         \
        return onerr;                                                                     \
    }

// Cost-model MLP (8 -> 64 -> 64 -> 1, binary32), see mlp.hip.
constexpr int MLP_NP = 4801;
size_t mlp_scratch_floats();
hipError_t launch_mlp_forward(const float* params, const float* X, int n, float* yhat, hipStream_t s);
hipError_t launch_mlp_grad(const float* params, const float* X, const float* y, const int* rows, int n,
                           float* scratch, float* grad, float* loss, hipStream_t s);
hipError_t launch_mlp_train(float* params, float* m, float* v, const float* X, const float* y, const int* order,
                            int n, int epochs, int bsz, int step0, float lr, float beta1, float beta2, float eps,
                            float* scratch, float* loss_out, hipStream_t s);

// Tiled executors, one per stencil kind.  b = {b_t, spatial sizes outer..inner}.
// *_supported: is the tile shape runnable; launch_*: one block per queue entry.
bool tiled1d_supported(const int* b);
hipError_t launch_tiled1d(int dtype, const int* b, const TiledLaunch& L, int grid_cap, hipStream_t s);
bool tiled2d_supported(const int* b);
hipError_t launch_tiled2d(int dtype, const int* b, const TiledLaunch& L, int grid_cap, hipStream_t s);
bool tiled3d_supported(const int* b, int lds_elem);
hipError_t launch_tiled3d(int dtype, const int* b, const TiledLaunch& L, int grid_cap, hipStream_t s);

}  // namespace pcot
