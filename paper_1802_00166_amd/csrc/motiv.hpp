// Executor of the appendix's motivating 1D program (motiv1d.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace pcot {

// b = {b_t, b_x} (skewed tiles of the 1D nest).
size_t motiv_lds_bytes(const int* b);
bool motiv_supported(const int* b);
// Y[0..T], Z[0..T] (the boundary statements' single-assignment arrays) and
// out[0] = Y[T], out[N-1] = Z[T].
hipError_t launch_motiv_boundary(const double* A, double* Y, double* Z, double* out, int N, int T, hipStream_t s);
// One untiled step t -> t+1 of the interior.
hipError_t launch_motiv_step(const double* src, double* dst, const double* Y, const double* Z, int N, int t,
                             hipStream_t s);
// The interior under a tiled / recursive plan (problem buffers: in = u_0,
// buf[t mod 2] = u_t).
hipError_t launch_motiv_tiles(const int* b, const TiledLaunch& L, const double* Y, const double* Z, hipStream_t s);

}  // namespace pcot
