// Untiled reference schedule (one sweep per time step), boundary copy and
// workspace clearing kernels.
#include "common.hpp"
#include "kernels.hpp"

namespace pcot {

// ------------------------------------------------------------- clearing ---
// A fill kernel rather than hipMemsetAsync so that launches stay safe to
// record into a HIP graph.
__global__ void k_fill_u32(unsigned* p, size_t n, unsigned v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

hipError_t launch_fill_u32(unsigned* p, size_t n, unsigned v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int block = 256;
    size_t grid = (n + block - 1) / block;
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)grid), dim3(block), 0, s, p, n, v);
    return hipGetLastError();
}

// Matrix dimensions 1 + (37 i mod pmax): a valid DP input for timing runs.
__global__ void k_fill_chain(long long* p, int n, long long pmax) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 1 + (long long)(((long long)i * 37) % pmax);
}

hipError_t launch_fill_chain(long long* p, int n, long long pmax, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_chain, dim3((n + 255) / 256), dim3(256), 0, s, p, n, pmax);
    return hipGetLastError();
}

__global__ void k_put_problem(TiledProblem* dst, TiledProblem v) {
    if (threadIdx.x == 0) *dst = v;
}

hipError_t launch_put_problem(TiledProblem* dst, const TiledProblem& v, hipStream_t s) {
    hipLaunchKernelGGL(k_put_problem, dim3(1), dim3(64), 0, s, dst, v);
    return hipGetLastError();
}

// Up to PUT_CHUNK descriptors per launch, passed by value (kernel arguments
// are recorded by value into a HIP graph, unlike a pageable host copy).
constexpr int PUT_CHUNK = 32;
struct ProblemChunk {
    TiledProblem p[PUT_CHUNK];
};
__global__ void k_put_problems(TiledProblem* dst, ProblemChunk c, int n) {
    if ((int)threadIdx.x < n) dst[threadIdx.x] = c.p[threadIdx.x];
}

hipError_t launch_put_problems(TiledProblem* dst, const TiledProblem* v, int n, hipStream_t s) {
    for (int i = 0; i < n; i += PUT_CHUNK) {
        ProblemChunk c;
        const int m = n - i < PUT_CHUNK ? n - i : PUT_CHUNK;
        for (int j = 0; j < m; ++j) c.p[j] = v[i + j];
        hipLaunchKernelGGL(k_put_problems, dim3(1), dim3(64), 0, s, dst + i, c, m);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ------------------------------------------------------- boundary copy ---
// Copies the outer face of a d-dimensional field (2d segments: each axis at
// index 0 and n-1; edges are copied more than once, with the same value).
template <typename S>
__device__ void copy_boundary_range(const S* __restrict__ src, S* __restrict__ dst0, S* __restrict__ dst1, int d,
                                    long long n0, long long n1, long long n2, long long start, long long stride) {
    const long long n[3] = {n0, n1, n2};
    long long seg_len[3];
    for (int a = 0; a < d; ++a) {
        long long c = 1;
        for (int b = 0; b < d; ++b)
            if (b != a) c *= n[b];
        seg_len[a] = c;
    }
    long long total = 0;
    for (int a = 0; a < d; ++a) total += 2 * seg_len[a];
    for (long long i = start; i < total; i += stride) {
        long long r = i;
        int a = 0;
        while (r >= 2 * seg_len[a]) { r -= 2 * seg_len[a]; ++a; }
        const int side = r >= seg_len[a];
        if (side) r -= seg_len[a];
        long long idx[3];
        for (int b = d - 1; b >= 0; --b) {
            if (b == a) { idx[b] = side ? n[b] - 1 : 0; continue; }
            idx[b] = r % n[b];
            r /= n[b];
        }
        long long off = 0;
        for (int b = 0; b < d; ++b) off = off * n[b] + idx[b];
        const S v = src[off];
        dst0[off] = v;
        if (dst1) dst1[off] = v;
    }
}

template <typename S>
__global__ void k_copy_boundary(const S* __restrict__ src, S* __restrict__ dst0, S* __restrict__ dst1,
                                int d, long long n0, long long n1, long long n2) {
    copy_boundary_range(src, dst0, dst1, d, n0, n1, n2, (long long)blockIdx.x * blockDim.x + threadIdx.x,
                        (long long)gridDim.x * blockDim.x);
}

// Batched form: blockIdx.y selects the problem; u_0's boundary goes to both
// of its buffers.
template <typename S>
__global__ void k_copy_boundary_batched(const TiledProblem* __restrict__ probs, int d) {
    const TiledProblem& P = probs[blockIdx.y];
    copy_boundary_range((const S*)P.in, (S*)P.buf0, (S*)P.buf1, d, P.n[0], P.n[1], P.n[2],
                        (long long)blockIdx.x * blockDim.x + threadIdx.x, (long long)gridDim.x * blockDim.x);
}

hipError_t launch_copy_boundary_batched(int dtype, const TiledProblem* probs, int nprob, int d, hipStream_t s) {
    if (nprob <= 0) return hipSuccess;
    const dim3 grid(64, (unsigned)nprob);
    switch (dtype) {
        case 0: hipLaunchKernelGGL(k_copy_boundary_batched<double>, grid, dim3(256), 0, s, probs, d); break;
        case 1: hipLaunchKernelGGL(k_copy_boundary_batched<float>, grid, dim3(256), 0, s, probs, d); break;
        default: hipLaunchKernelGGL(k_copy_boundary_batched<uint16_t>, grid, dim3(256), 0, s, probs, d); break;
    }
    return hipGetLastError();
}

template <typename S>
hipError_t launch_copy_boundary_t(const void* src, void* dst0, void* dst1, int d, const int64_t* n,
                                  hipStream_t s) {
    long long nn[3] = {1, 1, 1};
    long long total = 0;
    for (int a = 0; a < d; ++a) nn[a] = n[a];
    for (int a = 0; a < d; ++a) {
        long long c = 1;
        for (int b = 0; b < d; ++b)
            if (b != a) c *= nn[b];
        total += 2 * c;
    }
    const int block = 256;
    long long grid = (total + block - 1) / block;
    if (grid > 8192) grid = 8192;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_copy_boundary<S>, dim3((unsigned)grid), dim3(block), 0, s, (const S*)src,
                       (S*)dst0, (S*)dst1, d, nn[0], nn[1], nn[2]);
    return hipGetLastError();
}

hipError_t launch_copy_boundary(int dtype, const void* src, void* dst0, void* dst1, int d,
                                const int64_t* n, hipStream_t s) {
    switch (dtype) {
        case 0: return launch_copy_boundary_t<double>(src, dst0, dst1, d, n, s);
        case 1: return launch_copy_boundary_t<float>(src, dst0, dst1, d, n, s);
        default: return launch_copy_boundary_t<uint16_t>(src, dst0, dst1, d, n, s);
    }
}

// ------------------------------------------------------- naive sweeps ---
// One time step over the interior: dst = step(src).  Each thread updates
// VX consecutive points along the innermost axis.
template <typename S>
__global__ void __launch_bounds__(256) k_step1d(const S* __restrict__ src, S* __restrict__ dst, int n) {
    using A = typename Tr<S>::A;
    const int x = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    if (x > n - 2) return;
    const A v = jac1(Tr<S>::ld(src + x - 1), Tr<S>::ld(src + x), Tr<S>::ld(src + x + 1));
    Tr<S>::st(dst + x, v);
}

template <typename S>
__global__ void __launch_bounds__(256) k_step2d(const S* __restrict__ src, S* __restrict__ dst, int ny, int nx) {
    using A = typename Tr<S>::A;
    const int x = 1 + blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = 1 + blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x > nx - 2 || y > ny - 2) return;
    const size_t p = (size_t)y * nx + x;
    const A c = Tr<S>::ld(src + p);
    const A nn = Tr<S>::ld(src + p - nx);
    const A ss = Tr<S>::ld(src + p + nx);
    const A e = Tr<S>::ld(src + p + 1);
    const A w = Tr<S>::ld(src + p - 1);
    Tr<S>::st(dst + p, jac2(c, nn, ss, e, w));
}

template <typename S>
__global__ void __launch_bounds__(256) k_step3d(const S* __restrict__ src, S* __restrict__ dst, int nz, int ny, int nx) {
    using A = typename Tr<S>::A;
    const int x = 1 + blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = 1 + blockIdx.y * 4 + (threadIdx.x >> 6);
    const int z = 1 + blockIdx.z;
    if (x > nx - 2 || y > ny - 2) return;
    const size_t py = nx, pz = (size_t)ny * nx;
    const size_t p = (size_t)z * pz + (size_t)y * py + x;
    const A u = Tr<S>::ld(src + p);
    const A v = heat3(u, Tr<S>::ld(src + p + 1), Tr<S>::ld(src + p - 1), Tr<S>::ld(src + p + py),
                      Tr<S>::ld(src + p - py), Tr<S>::ld(src + p + pz), Tr<S>::ld(src + p - pz));
    Tr<S>::st(dst + p, v);
}

template <typename S>
hipError_t launch_step_t(int kind, const void* src, void* dst, const int64_t* n, hipStream_t s) {
    if (kind == 1) {
        const int len = (int)n[0];
        hipLaunchKernelGGL(k_step1d<S>, dim3((unsigned)((len - 2 + 255) / 256)), dim3(256), 0, s,
                           (const S*)src, (S*)dst, len);
    } else if (kind == 2) {
        const int ny = (int)n[0], nx = (int)n[1];
        dim3 grid((unsigned)((nx - 2 + 63) / 64), (unsigned)((ny - 2 + 3) / 4));
        hipLaunchKernelGGL(k_step2d<S>, grid, dim3(256), 0, s, (const S*)src, (S*)dst, ny, nx);
    } else {
        const int nz = (int)n[0], ny = (int)n[1], nx = (int)n[2];
        dim3 grid((unsigned)((nx - 2 + 63) / 64), (unsigned)((ny - 2 + 3) / 4), (unsigned)(nz - 2));
        hipLaunchKernelGGL(k_step3d<S>, grid, dim3(256), 0, s, (const S*)src, (S*)dst, nz, ny, nx);
    }
    return hipGetLastError();
}

hipError_t launch_step(int kind, int dtype, const void* src, void* dst, const int64_t* n, hipStream_t s) {
    switch (dtype) {
        case 0: return launch_step_t<double>(kind, src, dst, n, s);
        case 1: return launch_step_t<float>(kind, src, dst, n, s);
        default: return launch_step_t<uint16_t>(kind, src, dst, n, s);
    }
}

}  // namespace pcot
