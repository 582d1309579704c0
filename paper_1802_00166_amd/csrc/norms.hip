// Error norms of a stencil result against a binary64 reference, reduced in
// binary64 on the device in a fixed order (two passes: per-block partials,
// then one block over the partials), so repeated calls give identical bits.
#include "common.hpp"
#include "kernels.hpp"

#include <mutex>

namespace pcot {

namespace {

constexpr int NB = 256;   // threads per block
constexpr int NG = 1024;  // blocks of the first pass

template <typename S>
__device__ __forceinline__ double as_f64(const S* x, long long i) {
    return (double)Tr<S>::ld(x + i);
}

// Block-wide reduction of four values (max, max, sum, sum) in a fixed tree.
__device__ void block_reduce4(double v[4], double* sh) {
    const int t = threadIdx.x;
    for (int q = 0; q < 4; ++q) sh[q * NB + t] = v[q];
    __syncthreads();
    for (int w = NB / 2; w > 0; w >>= 1) {
        if (t < w) {
            sh[0 * NB + t] = fmax(sh[0 * NB + t], sh[0 * NB + t + w]);
            sh[1 * NB + t] = fmax(sh[1 * NB + t], sh[1 * NB + t + w]);
            sh[2 * NB + t] = sh[2 * NB + t] + sh[2 * NB + t + w];
            sh[3 * NB + t] = sh[3 * NB + t] + sh[3 * NB + t + w];
        }
        __syncthreads();
    }
    for (int q = 0; q < 4; ++q) v[q] = sh[q * NB];
}

template <typename S>
__global__ void __launch_bounds__(NB) k_norms_pass1(const S* __restrict__ x, const double* __restrict__ r, int d,
                                                    long long n0, long long n1, long long n2, double* part) {
    __shared__ double sh[4 * NB];
    // interior points are enumerated as a (n0-2) x (n1-2) x (n2-2) box
    const long long m0 = n0 - 2, m1 = d >= 2 ? n1 - 2 : 1, m2 = d >= 3 ? n2 - 2 : 1;
    const long long total = m0 * m1 * m2;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (long long q = (long long)blockIdx.x * NB + threadIdx.x; q < total; q += (long long)NG * NB) {
        long long a = q, i0, i1 = 0, i2 = 0;
        if (d == 3) { i2 = a % m2; a /= m2; }
        if (d >= 2) { i1 = a % m1; a /= m1; }
        i0 = a;
        long long off;
        if (d == 1) off = 1 + i0;
        else if (d == 2) off = (1 + i0) * n1 + (1 + i1);
        else off = ((1 + i0) * n1 + (1 + i1)) * n2 + (1 + i2);
        const double rv = r[off], e = as_f64(x, off) - rv;
        v[0] = fmax(v[0], fabs(e));
        v[1] = fmax(v[1], fabs(rv));
        v[2] += e * e;
        v[3] += rv * rv;
    }
    block_reduce4(v, sh);
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) part[blockIdx.x * 4 + k] = v[k];
}

__global__ void __launch_bounds__(NB) k_norms_pass2(const double* __restrict__ part, double* out) {
    __shared__ double sh[4 * NB];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < NG; b += NB) {
        v[0] = fmax(v[0], part[b * 4 + 0]);
        v[1] = fmax(v[1], part[b * 4 + 1]);
        v[2] += part[b * 4 + 2];
        v[3] += part[b * 4 + 3];
    }
    block_reduce4(v, sh);
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) out[k] = v[k];
}

}  // namespace

size_t norms_scratch_bytes() { return (size_t)(NG * 4 + 4) * sizeof(double); }

hipError_t launch_norms(int dtype, int d, const int64_t* n, const void* x, const double* r, double* scratch,
                        hipStream_t s) {
    return launch_norms_to(dtype, d, n, x, r, scratch, scratch + NG * 4, s);
}

hipError_t launch_norms_to(int dtype, int d, const int64_t* n, const void* x, const double* r, double* scratch,
                           double* result, hipStream_t s) {
    const long long n0 = n[0], n1 = d >= 2 ? n[1] : 1, n2 = d >= 3 ? n[2] : 1;
    switch (dtype) {
        case 0: hipLaunchKernelGGL(k_norms_pass1<double>, dim3(NG), dim3(NB), 0, s, (const double*)x, r, d, n0, n1, n2, scratch); break;
        case 1: hipLaunchKernelGGL(k_norms_pass1<float>, dim3(NG), dim3(NB), 0, s, (const float*)x, r, d, n0, n1, n2, scratch); break;
        default: hipLaunchKernelGGL(k_norms_pass1<uint16_t>, dim3(NG), dim3(NB), 0, s, (const uint16_t*)x, r, d, n0, n1, n2, scratch); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_norms_pass2, dim3(1), dim3(NB), 0, s, scratch, result);
    return hipGetLastError();
}

// Allocation-free variant's scratch: the first pass's partials (NG blocks x 4
// values, every slot rewritten by every call, so nothing needs clearing).
// One copy per GPU, held until the process ends.  Its host-side name is not a
// device address: host code uses the address looked up per device below.
__device__ __align__(256) double scratch[NG * 4];
namespace {
constexpr int MAX_DEV = 64;
std::mutex g_static_mu;
double* g_static_ptr[MAX_DEV] = {};
}  // namespace

size_t norms_static_scratch_bytes() { return sizeof(double) * NG * 4; }

hipError_t norms_static_scratch(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_static_ptr[dev] = (double*)p;
    }
    *out = g_static_ptr[dev];
    return hipSuccess;
}

}  // namespace pcot
