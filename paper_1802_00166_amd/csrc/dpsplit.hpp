// Parenthesization pass of the matrix-chain DP (dp_split.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace pcot {

// split (device, N x N int64) from the final costs C (device, N x N int64)
// and dimensions p (device, N + 1 int64).
hipError_t launch_dp_split(const long long* p, const long long* C, long long* split, int N, hipStream_t s);

}  // namespace pcot
