// Front executor for nests with dependences inside a time step: the in-place
// Gauss-Seidel-2D stencil and FDTD-2D after the embedding transformation.
//
// Gauss-Seidel-2D (kind 4), in place, sweep t visits the interior in
// lexicographic order:  u[y][x] = 0.2*((((c + n) + s) + e) + w)  with n, w of
// sweep t and c, s, e of sweep t-1.  Dependence distances in (t, y, x):
// (0,1,0), (0,0,1), (1,-1,0), (1,0,-1), (1,0,0) (flow, anti and output alike).
// After the skew (t, y, x) -> (t, jy = y + t, jx = x + t) they become
// (0,1,0), (0,0,1), (1,0,1), (1,1,0), (1,1,1): the nest is fully permutable
// (Section 3: tiling legality; the paper's point that Gauss-Seidel style
// dependences fit its framework, Section 6.2), so the skewed box tiles and
// their orders are those of the Jacobi stencils.  Inside a tile every
// dependence increases jy + jx, so the points of one front jy + jx = theta
// (all levels of the tile together) are independent.
//
// FDTD-2D (kind 5): the time loop holds three loop nests (ey, ex, hz
// updates; an imperfect nest).  The embedding transformation (Section 4.4)
// brings the three statements into one (t, i, j) nest with guards; the hz
// statement is shifted by (0, 1, 1): iteration (t, i, j) runs
//   S1 ey[i][j]      -= CE (hz[i][j] - hz[i-1][j])              if 1 <= i
//   S2 ex[i][j]      += CE (hz[i][j] - hz[i][j-1])              if 1 <= j
//   S3 hz[i-1][j-1]  -= CH ((ey[i][j-1] - ey[i-1][j-1]) - (ex[i-1][j] - ex[i-1][j-1]))
//                                                               if 1 <= i, 1 <= j
// for 0 <= i < ny, 0 <= j < nx.  With the shift every dependence inside a
// step has distance (0, a, b), a, b >= 0, and those across steps (1, a, b)
// with a, b >= -1, so the same skew makes the nest fully permutable with all
// distances in {0,1}^3; inside a tile t + jy + jx increases along every
// dependence and defines the fronts.  (The planner sees the nest as a
// stencil on (ny + 2) x (nx + 2) cells, so skewed jy = i + t + 1.)
//
// A block copies the tile's footprint (every cell its points read or write,
// for all levels) from global memory to LDS, runs the fronts in LDS with one
// barrier per front, and writes back exactly the cells the tile updates
// (their last values).  In-place execution is exact: a tile starts only when
// its predecessors are done, so every cell it reads holds the value the
// sequential program would read; cells it copies but does not own are never
// written back.
#include "bufio.hpp"
#include "common.hpp"
#include "front.hpp"

namespace pcot {

namespace {

constexpr int NT = 512;  // threads per block
constexpr int NB_GS = 8, NB_FDTD = 4;  // copy-in loads per thread and field in flight together
constexpr double FDTD_CE = 0.25, FDTD_CH = 0.5;

struct Geo {
    int t0, nt, t1, Y0, X0, by, bx;
    int oy, ox, Hy, Hx;  // footprint origin (array indices) and extents, Hx padded
};

__host__ __device__ inline int pad_row(int w) {
    // row stride in doubles with (stride - 1) = 1 mod 32: a front steps one
    // row down and one column left, so consecutive threads hit different banks
    return w + ((33 - (w - 1) % 32) % 32);
}

__device__ __forceinline__ Geo geo_of(const TiledProblem& P, const int* k, int off) {
    Geo g;
    g.by = P.b[1];
    g.bx = P.b[2];
    g.t0 = k[0] * P.b[0];
    g.nt = min(P.b[0], P.T - g.t0);
    g.t1 = g.t0 + g.nt - 1;
    g.Y0 = 1 + k[1] * g.by;
    g.X0 = 1 + k[2] * g.bx;
    g.oy = g.Y0 - g.t1 - 1 - off;
    g.ox = g.X0 - g.t1 - 1 - off;
    g.Hy = g.by + g.nt + 1;
    g.Hx = pad_row(g.bx + g.nt + 1);
    return g;
}

// Does the tile update cell (a, b) of the skewed-minus-offset grid, i.e. is
// there a level t in [t0, t1] with jy = a + t + off in [Y0, Y0 + by) and
// jx = b + t + off in [X0, X0 + bx)?
__device__ __forceinline__ bool tile_owns(const Geo& g, int a, int b, int off) {
    const int lo = max(g.t0, max(g.Y0 - a - off, g.X0 - b - off));
    const int hi = min(g.t1, min(g.Y0 + g.by - 1 - a - off, g.X0 + g.bx - 1 - b - off));
    return lo <= hi;
}

__device__ void exec_gs(const TiledProblem& P, const int* k, double* lds) {
    const int ny = P.n[0], nx = P.n[1];
    const Geo g = geo_of(P, k, 0);
    const uint32_t bytes = (uint32_t)ny * (uint32_t)nx * 8;
    const rsrc_t rf = make_rsrc(uptr(P.buf0), bytes);
    const int cells = g.Hy * g.Hx;
    // copy-in: a batch of loads in flight per thread before its LDS stores
    // (a load followed at once by its store would cost a round trip each)
    for (int q0 = threadIdx.x; q0 < cells; q0 += NT * NB_GS) {
        double v[NB_GS];
#pragma unroll
        for (int b = 0; b < NB_GS; ++b) {
            const int q = q0 + b * NT;
            const int y = g.oy + q / g.Hx, x = g.ox + q % g.Hx;
            const bool in = q < cells && y >= 0 && y < ny && x >= 0 && x < nx;
            v[b] = IO<double>::ld(rf, in ? (y * nx + x) * 8 : OOB);
        }
#pragma unroll
        for (int b = 0; b < NB_GS; ++b)
            if (q0 + b * NT < cells) lds[q0 + b * NT] = v[b];
    }
    __syncthreads();
    const int npair = g.nt * g.by;
    for (int th = g.Y0 + g.X0; th <= g.Y0 + g.by - 1 + g.X0 + g.bx - 1; ++th) {
        for (int q = threadIdx.x; q < npair; q += NT) {
            const int t = g.t0 + q / g.by, jy = g.Y0 + q % g.by, jx = th - jy;
            const int y = jy - t, x = jx - t;
            if (jx >= g.X0 && jx < g.X0 + g.bx && y >= 1 && y <= ny - 2 && x >= 1 && x <= nx - 2) {
                double* u = lds + (y - g.oy) * g.Hx + (x - g.ox);
                u[0] = 0.2 * ((((u[0] + u[-g.Hx]) + u[g.Hx]) + u[1]) + u[-1]);
            }
        }
        __syncthreads();
    }
    for (int q = threadIdx.x; q < cells; q += NT) {
        const int y = g.oy + q / g.Hx, x = g.ox + q % g.Hx;
        const bool own = y >= 1 && y <= ny - 2 && x >= 1 && x <= nx - 2 && tile_owns(g, y, x, 0);
        IO<double>::st(rf, own ? (y * nx + x) * 8 : OOB, lds[q]);
    }
}

__device__ void exec_fdtd(const TiledProblem& P, const int* k, double* lds) {
    // planner extents are (ny + 2) x (nx + 2)
    const int ny = P.n[0] - 2, nx = P.n[1] - 2;
    const Geo g = geo_of(P, k, 1);
    const uint32_t bytes = (uint32_t)ny * (uint32_t)nx * 8;
    const rsrc_t rex = make_rsrc(uptr(P.buf0), bytes), rey = make_rsrc(uptr(P.buf1), bytes),
                 rhz = make_rsrc(uptr(P.in), bytes);
    const int cells = g.Hy * g.Hx;
    double* ex = lds;
    double* ey = lds + cells;
    double* hz = lds + 2 * cells;
    for (int q0 = threadIdx.x; q0 < cells; q0 += NT * NB_FDTD) {
        double vx[NB_FDTD], vy[NB_FDTD], vh[NB_FDTD];
#pragma unroll
        for (int b = 0; b < NB_FDTD; ++b) {
            const int q = q0 + b * NT;
            const int i = g.oy + q / g.Hx, j = g.ox + q % g.Hx;
            const int o = (q < cells && i >= 0 && i < ny && j >= 0 && j < nx) ? (i * nx + j) * 8 : OOB;
            vx[b] = IO<double>::ld(rex, o);
            vy[b] = IO<double>::ld(rey, o);
            vh[b] = IO<double>::ld(rhz, o);
        }
#pragma unroll
        for (int b = 0; b < NB_FDTD; ++b) {
            const int q = q0 + b * NT;
            if (q < cells) {
                ex[q] = vx[b];
                ey[q] = vy[b];
                hz[q] = vh[b];
            }
        }
    }
    __syncthreads();
    const int npair = g.nt * g.by;
    const int th0 = g.t0 + g.Y0 + g.X0, th1 = g.t1 + g.Y0 + g.by - 1 + g.X0 + g.bx - 1;
    for (int th = th0; th <= th1; ++th) {
        for (int q = threadIdx.x; q < npair; q += NT) {
            const int t = g.t0 + q / g.by, jy = g.Y0 + q % g.by, jx = th - t - jy;
            const int i = jy - t - 1, j = jx - t - 1;
            if (jx >= g.X0 && jx < g.X0 + g.bx && i >= 0 && i < ny && j >= 0 && j < nx) {
                const int c = (i - g.oy) * g.Hx + (j - g.ox);
                if (i >= 1) ey[c] = ey[c] - FDTD_CE * (hz[c] - hz[c - g.Hx]);
                if (j >= 1) ex[c] = ex[c] + FDTD_CE * (hz[c] - hz[c - 1]);
                if (i >= 1 && j >= 1) {
                    const int d = c - g.Hx - 1;  // cell (i-1, j-1)
                    hz[d] = hz[d] - FDTD_CH * ((ey[d + g.Hx] - ey[d]) - (ex[d + 1] - ex[d]));
                }
            }
        }
        __syncthreads();
    }
    for (int q = threadIdx.x; q < cells; q += NT) {
        const int i = g.oy + q / g.Hx, j = g.ox + q % g.Hx;
        const bool in = i >= 0 && i < ny && j >= 0 && j < nx;
        const int o = (i * nx + j) * 8;
        // ey(i, j), ex(i, j) at iteration (t, i, j); hz(i, j) at (t, i+1, j+1)
        const bool oe = in && tile_owns(g, i, j, 1);
        const bool oh = in && i <= ny - 2 && j <= nx - 2 && tile_owns(g, i + 1, j + 1, 1);
        IO<double>::st(rey, oe && i >= 1 ? o : OOB, ey[q]);
        IO<double>::st(rex, oe && j >= 1 ? o : OOB, ex[q]);
        IO<double>::st(rhz, oh ? o : OOB, hz[q]);
    }
}

template <int KIND>
__global__ void __launch_bounds__(NT) k_front2d(TiledLaunch Lc) {
    extern __shared__ double lds[];
    __shared__ int s_tk, s_go;
    run_queued_tile<2, true>(Lc, &s_tk, &s_go, [&](const TiledProblem& P, const int* k) {
        if constexpr (KIND == 4) exec_gs(P, k, lds);
        else exec_fdtd(P, k, lds);
    });
}

__global__ void k_fdtd_ey(double* ey, const double* hz, int ny, int nx) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long long)(ny - 1) * nx) return;
    const long long c = q + nx;  // rows 1 .. ny-1
    ey[c] = ey[c] - FDTD_CE * (hz[c] - hz[c - nx]);
}
__global__ void k_fdtd_ex(double* ex, const double* hz, int ny, int nx) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long long)ny * (nx - 1)) return;
    const long long i = q / (nx - 1), j = 1 + q % (nx - 1);
    const long long c = i * nx + j;
    ex[c] = ex[c] + FDTD_CE * (hz[c] - hz[c - 1]);
}
__global__ void k_fdtd_hz(double* hz, const double* ex, const double* ey, int ny, int nx) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long long)(ny - 1) * (nx - 1)) return;
    const long long i = q / (nx - 1), j = q % (nx - 1);
    const long long c = i * nx + j;
    hz[c] = hz[c] - FDTD_CH * ((ey[c + nx] - ey[c]) - (ex[c + 1] - ex[c]));
}

}  // namespace

size_t front2d_lds_bytes(int kind, const int* b) {
    const int Hy = b[1] + b[0] + 1, Hx = pad_row(b[2] + b[0] + 1);
    return (size_t)(kind == 5 ? 3 : 1) * Hy * Hx * sizeof(double);
}

bool front2d_supported(int kind, int dtype, const int* b) {
    if (dtype != 0 || (kind != 4 && kind != 5)) return false;
    if (b[0] < 1 || b[1] < 2 || b[2] < 2 || b[0] > 256 || b[1] > 1024 || b[2] > 1024) return false;
    return front2d_lds_bytes(kind, b) <= 160 * 1024 - 256;
}

hipError_t launch_front2d(int kind, const int* b, const TiledLaunch& L, hipStream_t s) {
    if (L.nq <= 0) return hipSuccess;
    const size_t lds = front2d_lds_bytes(kind, b);
    if (kind == 4) {
        if (lds > 65536) {
            const hipError_t e = hipFuncSetAttribute((const void*)k_front2d<4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_front2d<4>, dim3(L.nq), dim3(NT), lds, s, L);
    } else {
        if (lds > 65536) {
            const hipError_t e = hipFuncSetAttribute((const void*)k_front2d<5>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_front2d<5>, dim3(L.nq), dim3(NT), lds, s, L);
    }
    return hipGetLastError();
}

hipError_t launch_fdtd2d_step(double* ex, double* ey, double* hz, int ny, int nx, hipStream_t s) {
    const int B = 256;
    auto nb = [&](long long n) { return dim3((unsigned)((n + B - 1) / B)); };
    // a statement with an empty range (one row or one column) launches nothing
    if (ny > 1) hipLaunchKernelGGL(k_fdtd_ey, nb((long long)(ny - 1) * nx), dim3(B), 0, s, ey, hz, ny, nx);
    if (nx > 1) hipLaunchKernelGGL(k_fdtd_ex, nb((long long)ny * (nx - 1)), dim3(B), 0, s, ex, hz, ny, nx);
    if (ny > 1 && nx > 1)
        hipLaunchKernelGGL(k_fdtd_hz, nb((long long)(ny - 1) * (nx - 1)), dim3(B), 0, s, hz, ex, ey, ny, nx);
    return hipGetLastError();
}

}  // namespace pcot
