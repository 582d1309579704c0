// Front executor: skewed box tiles of nests whose dependences include ones
// inside a time step, run point by point in wavefronts of the tile (the
// in-place Gauss-Seidel-2D stencil and the three-statement FDTD-2D update
// after the embedding transformation).  Same tile grid, queue and
// dependency counters as the Jacobi executors (kernels.hpp).
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace pcot {

// kind 4: Gauss-Seidel-2D (field in P.buf0, updated in place);
// kind 5: FDTD-2D (ex in P.buf0, ey in P.buf1, hz in P.in, all in place).
// b = {b_t, b_y, b_x} in skewed coordinates.
size_t front2d_lds_bytes(int kind, const int* b);
bool front2d_supported(int kind, int dtype, const int* b);
hipError_t launch_front2d(int kind, const int* b, const TiledLaunch& L, hipStream_t s);
// One untiled FDTD-2D time step (three kernels: ey, ex, hz), in place.
hipError_t launch_fdtd2d_step(double* ex, double* ey, double* hz, int ny, int nx, hipStream_t s);

}  // namespace pcot
