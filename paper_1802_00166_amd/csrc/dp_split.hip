// Optimal parenthesization of the matrix chain from its final cost table:
// for every cell (a, c), a < c (0-based; A_{a+1}..A_{c+1}), the smallest
// split k' in [a, c) with C[a][k'] + C[k'+1][c] + p[a] p[k'+1] p[c+1] equal to
// C[a][c] (the smallest-k tie-break of a sequential scan with a strict
// comparison).  Reported 1-based, k = k' + 1 (A_k | A_{k+1}); 0 on and below
// the diagonal.  The cost table is exact and final, so this pass is
// independent of the order in which the DP reduced its splits.
//
// Lanes of a wave take 64 consecutive columns c of one row a, so C[k'+1][c]
// is one coalesced row segment per step and C[a][k'], p[k'+1] are the same
// for all lanes; a wave stops once every lane has found its split.
#include <hip/hip_runtime.h>
#include <cstdint>

#include "dpsplit.hpp"

namespace pcot {

namespace {

__global__ void __launch_bounds__(256) k_dp_split(const long long* __restrict__ p, const long long* __restrict__ C,
                                                  long long* __restrict__ split, int N) {
    const int a = blockIdx.y;
    const int c = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 64 + (threadIdx.x & 63);
    const bool cell = c < N && c > a;
    if (c < N && c <= a) split[(size_t)a * N + c] = 0;
    const long long target = cell ? C[(size_t)a * N + c] : 0;
    const long long wa = p[a] * (cell ? p[c + 1] : 0);
    long long found = cell ? -1 : 0;
    const int kend = min(N - 1, (blockIdx.x * 4 + (int)(threadIdx.x >> 6)) * 64 + 63);  // largest c of the wave, capped
    for (int k = a; k < kend; ++k) {
        if (__ballot(found < 0) == 0) break;
        if (found < 0 && k < c) {
            const long long q = C[(size_t)a * N + k] + C[(size_t)(k + 1) * N + c] + wa * p[k + 1];
            if (q == target) found = k + 1;
        }
    }
    if (cell) split[(size_t)a * N + c] = found < 0 ? 0 : found;
}

}  // namespace

hipError_t launch_dp_split(const long long* p, const long long* C, long long* split, int N, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    const dim3 grid((unsigned)((N + 255) / 256), (unsigned)N);
    hipLaunchKernelGGL(k_dp_split, grid, dim3(256), 0, s, p, C, split, N);
    return hipGetLastError();
}

}  // namespace pcot
