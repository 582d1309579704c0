// Untiled Jacobi-1D sweep held in one CU's LDS (resident1d.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace pcot {

// Whether both time levels of an n-point field fit in one block's LDS.
bool resident1d_fits(int dtype, int64_t n);
// All T steps in one block; out receives u_T (boundary included).
hipError_t launch_resident1d(int dtype, const void* in, void* out, int n, int T, hipStream_t s);

}  // namespace pcot
