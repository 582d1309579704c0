// The untiled Jacobi-1D sweep for fields that fit in one CU's LDS: one block
// keeps both time levels of the whole field in LDS for all T steps (one
// barrier per step) and writes u_T once.  Each point uses the same operation
// order as the per-step kernels, so the bits are those of every other
// schedule.  A 4096-point f64 field is 32 KiB: launching one kernel per step
// would spend the run in launch gaps.
#include "common.hpp"
#include "resident.hpp"

namespace pcot {

namespace {

constexpr int NT = 1024;

template <typename S>
__global__ void __launch_bounds__(NT) k_resident1d(const S* __restrict__ in, S* __restrict__ out, int n, int T) {
    using A = typename Tr<S>::A;
    extern __shared__ char raw[];
    A* a = reinterpret_cast<A*>(raw);
    A* b = a + n;
    for (int i = threadIdx.x; i < n; i += NT) a[i] = b[i] = Tr<S>::ld(in + i);
    __syncthreads();
    for (int t = 0; t < T; ++t) {
        for (int i = 1 + threadIdx.x; i < n - 1; i += NT) b[i] = Tr<S>::rnd(jac1(a[i - 1], a[i], a[i + 1]));
        __syncthreads();
        A* c = a;
        a = b;
        b = c;
    }
    for (int i = threadIdx.x; i < n; i += NT) Tr<S>::st(out + i, a[i]);
}

template <typename S>
hipError_t launch_t(const void* in, void* out, int n, int T, hipStream_t s) {
    const size_t lds = 2 * (size_t)n * sizeof(typename Tr<S>::A);
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute((const void*)k_resident1d<S>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_resident1d<S>, dim3(1), dim3(NT), lds, s, (const S*)in, (S*)out, n, T);
    return hipGetLastError();
}

}  // namespace

bool resident1d_fits(int dtype, int64_t n) {
    const int64_t es = dtype == 0 ? 8 : 4;  // arithmetic type held in LDS
    return n >= 3 && 2 * n * es <= 160 * 1024 - 256;
}

hipError_t launch_resident1d(int dtype, const void* in, void* out, int n, int T, hipStream_t s) {
    switch (dtype) {
        case 0: return launch_t<double>(in, out, n, T, s);
        case 1: return launch_t<float>(in, out, n, T, s);
        default: return launch_t<uint16_t>(in, out, n, T, s);
    }
}

}  // namespace pcot
