// The appendix's motivating 1D program (Memory Allocation, Fig. motiv) under
// the tiled and recursive schedules, with the schedule-independent memory
// allocation the appendix derives:
//   S1  X[t][i]   = f(X[t-1][i-1], X[t-1][i], X[t-1][i+1], X[t-1][0])   1 <= i <= N-2
//   S2  X[t][0]   = g(X[t-1][0]),   S3  X[t][N-1] = g(X[t-1][N-1])
// with f(a, b, c, d) = 0.25 (((a + b) + c) + d), g(y) = 0.5 y + 0.25.
// The dependence of every S1 point on S2 of the previous step is affine and
// many-to-one, and with the original two-buffer storage it brings
// memory-based dependences that forbid time tiling.  The affine split gives
// the values of S2 (and S3) a single-assignment array each, Y[t] and Z[t];
// S1 keeps the two-buffer allocation X[t mod 2] (its dependences are uniform,
// and radius 1 makes the buffers a universal occupancy vector).  Memory:
// 2N + 2(T+1) values instead of the full expansion's (T+1) N.
//
// Y and Z depend only on themselves, so one thread writes them first; the
// interior then runs as skewed tiles from the device queue (any order the
// planner emits), reading Y[t] / Z[t] wherever the program reads the
// boundary cells.  A tile keeps two levels in LDS: every needed level-t0
// value and the two-point faces of every level (written by the tile to its
// left, a predecessor) are loaded at the start, the levels run in LDS with
// one barrier each, and the tile stores its two rightmost points of every
// level and its top level.
#include "bufio.hpp"
#include "common.hpp"
#include "motiv.hpp"

namespace pcot {

namespace {

constexpr int NT = 256;

__device__ __forceinline__ double mf(double a, double b, double c, double d) { return 0.25 * (((a + b) + c) + d); }
__device__ __forceinline__ double mg(double y) { return 0.5 * y + 0.25; }

__global__ void k_motiv_boundary(const double* A, double* Y, double* Z, double* out, int N, int T) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double y = A[0], z = A[N - 1];
    Y[0] = y;
    Z[0] = z;
    for (int t = 1; t <= T; ++t) {
        y = mg(y);
        z = mg(z);
        Y[t] = y;
        Z[t] = z;
    }
    out[0] = y;
    out[N - 1] = z;
}

// One untiled step t -> t+1 of S1 (interior) with the boundary from Y, Z.
__global__ void k_motiv_step(const double* src, double* dst, const double* Y, const double* Z, int N, int t) {
    const int i = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    if (i > N - 2) return;
    const double left = i == 1 ? Y[t] : src[i - 1];
    const double right = i == N - 2 ? Z[t] : src[i + 1];
    dst[i] = mf(left, src[i], right, Y[t]);
}

__device__ void exec_motiv(const TiledProblem& P, const int* k, const double* Y, const double* Z, double* lds) {
    const int N = P.n[0], bx = P.b[1];
    const int t0 = k[0] * P.b[0];
    const int nt = min(P.b[0], P.T - t0);
    const int t1 = t0 + nt - 1;
    const int J0 = 1 + k[1] * bx;        // skewed start: j = i + t
    const int ox = J0 - t1 - 1;          // first array index held
    const int W = bx + nt + 2;           // held width
    double* cur = lds;
    double* nxt = lds + W;
    double* face = lds + 2 * W;          // face[2 * l + q]: u_{t0+l} at index J0 - t0 - l - 1 + q
    const uint32_t bytes = (uint32_t)N * 8;
    const uintptr_t pin = (uintptr_t)uptr(P.in), pb0 = (uintptr_t)uptr(P.buf0), pb1 = (uintptr_t)uptr(P.buf1);
    auto src_of = [&](int t) { return make_rsrc(uptr((const void*)pick(pick(pb0, pb1, t), pin, t == 0)), bytes); };
    auto val = [&](int t, int x) -> double {  // u_t(x) from memory (boundary from Y, Z)
        if (x == 0) return Y[t];
        if (x == N - 1) return Z[t];
        return IO<double>::ld(src_of(t), (x >= 1 && x <= N - 2) ? x * 8 : OOB);
    };
    // level-t0 values over [J0 - t0 - 1, J0 + bx - t0 + 1), faces of later levels
    for (int q = threadIdx.x; q < W; q += NT) {
        const int x = ox + q;
        const bool need = x >= J0 - t0 - 1 && x < J0 + bx - t0 + 1 && x >= 0 && x < N;
        cur[q] = need ? val(t0, x) : 0.0;
    }
    // the faces' time steps differ between lanes, and a buffer descriptor
    // must be the same for the whole wave: both buffers are read (the other
    // offset out of range) and each lane keeps the one of its step's parity
    {
        const rsrc_t r0 = make_rsrc(uptr((const void*)pb0), bytes), r1 = make_rsrc(uptr((const void*)pb1), bytes);
        for (int q = threadIdx.x; q < 2 * nt; q += NT) {
            const int l = q / 2, x = J0 - t0 - l - 1 + (q % 2), t = t0 + l;
            double v = 0.0;
            if (l > 0 && x == 0) v = Y[t];
            else if (l > 0 && x == N - 1) v = Z[t];
            else if (l > 0) {
                const int o = (x >= 1 && x <= N - 2) ? x * 8 : OOB;
                const double a0 = IO<double>::ld(r0, (t & 1) ? OOB : o), a1 = IO<double>::ld(r1, (t & 1) ? o : OOB);
                v = (t & 1) ? a1 : a0;
            }
            face[q] = v;
        }
    }
    __syncthreads();
    for (int l = 0; l < nt; ++l) {
        const int t = t0 + l;
        if (l > 0) {  // the two points left of this level's range come from the left tile
            if (threadIdx.x < 2) {
                const int x = J0 - t - 1 + threadIdx.x;
                if (x >= ox) cur[x - ox] = face[2 * l + threadIdx.x];
            }
            __syncthreads();
        }
        const double d = Y[t];
        const rsrc_t dst = make_rsrc(uptr((const void*)pick(pb0, pb1, t + 1)), bytes);
        for (int q = threadIdx.x; q < bx; q += NT) {
            const int x = J0 + q - t;
            if (x >= 1 && x <= N - 2) {
                const int c = x - ox;
                const double left = x == 1 ? Y[t] : cur[c - 1];
                const double right = x == N - 2 ? Z[t] : cur[c + 1];
                const double v = mf(left, cur[c], right, d);
                nxt[c] = v;
                // stores: the two rightmost points of the level (the right
                // tile's faces) and the whole top level
                if (l == nt - 1 || q >= bx - 2) IO<double>::st(dst, x * 8, v);
            }
        }
        __syncthreads();
        double* tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
}

__global__ void __launch_bounds__(NT) k_motiv_tiles(TiledLaunch Lc, const double* Y, const double* Z) {
    extern __shared__ double lds[];
    __shared__ int s_tk, s_go;
    run_queued_tile<1, true>(Lc, &s_tk, &s_go,
                             [&](const TiledProblem& P, const int* k) { exec_motiv(P, k, Y, Z, lds); });
}

}  // namespace

size_t motiv_lds_bytes(const int* b) { return (size_t)(2 * (b[1] + b[0] + 2) + 2 * b[0]) * sizeof(double); }

bool motiv_supported(const int* b) {
    return b[0] >= 1 && b[0] <= 4096 && b[1] >= 2 && b[1] <= 8192 && motiv_lds_bytes(b) <= 160 * 1024 - 256;
}

hipError_t launch_motiv_boundary(const double* A, double* Y, double* Z, double* out, int N, int T, hipStream_t s) {
    hipLaunchKernelGGL(k_motiv_boundary, dim3(1), dim3(64), 0, s, A, Y, Z, out, N, T);
    return hipGetLastError();
}

hipError_t launch_motiv_step(const double* src, double* dst, const double* Y, const double* Z, int N, int t,
                             hipStream_t s) {
    if (N < 3) return hipSuccess;
    hipLaunchKernelGGL(k_motiv_step, dim3((N - 2 + 255) / 256), dim3(256), 0, s, src, dst, Y, Z, N, t);
    return hipGetLastError();
}

hipError_t launch_motiv_tiles(const int* b, const TiledLaunch& L, const double* Y, const double* Z, hipStream_t s) {
    if (L.nq <= 0) return hipSuccess;
    const size_t lds = motiv_lds_bytes(b);
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute((const void*)k_motiv_tiles, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_motiv_tiles, dim3(L.nq), dim3(NT), lds, s, L, Y, Z);
    return hipGetLastError();
}

}  // namespace pcot
