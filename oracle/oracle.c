/*
 * Oracle: plain, untiled CPU loop nests that define what the hot path computes.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * path.
 *
 * The paper's method (time-skewed single-level tiling, and its cache-oblivious
 * recursive decomposition; Sections 3-4 of the paper) only reorders the points
 * of a fully permutable loop nest.  So the result it must reproduce is the
 * plain definition: the untiled nest, time outermost, points in lexicographic
 * order, values held in two buffers indexed by t mod 2 (the two-buffer
 * storage of the 1D-Jacobi example in the appendix on schedule-independent
 * memory allocation).
 *
 * Update rules (one time step, interior points only; boundary cells are never
 * written and keep their input value):
 *   Jacobi-1D 3-point: u'[i]    = ((u[i-1] + u[i]) + u[i+1]) / 3
 *   Jacobi-2D 5-point: u'[y][x] = 0.2 * ((((c + n) + s) + e) + w)
 *                      c=u[y][x] n=u[y-1][x] s=u[y+1][x] e=u[y][x+1] w=u[y][x-1]
 *   Heat-3D 7-point:   u' = u + 0.125 * ((dx + dy) + dz),
 *                      dx = (u[x+1] - 2u) + u[x-1], likewise dy, dz
 * The operation order is exactly as written; the file is compiled with
 * -ffp-contract=off so no multiply-add is fused.  f64 and f32 variants use
 * the literals 3.0/0.2/0.125/2.0 of their own type.  The bf16 variant stores
 * bfloat16 bit patterns, widens each load exactly to f32, computes in f32 and
 * rounds every stored value to nearest-even bf16.
 *
 * Interval DP (matrix-chain / optimal parenthesization, the interval DP the
 * paper benchmarks as OSP): C[i][i] = 0,
 *   C[i][j] = min_{i<=k<j} C[i][k] + C[k+1][j] + p[i-1]*p[k]*p[j],
 * evaluated by increasing chain length in int64, ties broken toward the
 * smallest k.  Integer min/+ are exact, so any reordering of k (the
 * Guibas-Kung-Thompson reordering the paper applies to tile OSP) gives
 * identical values.
 *
 * The optional OpenMP pragma on the outermost spatial loop (or on i within a
 * DP diagonal) splits independent points across threads without changing any
 * operation, so the bits are identical at every thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------ threads --- */

void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n < 1) n = 1;
    omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------- bf16 storage --- */

static float bf16_load(uint16_t h) {
    uint32_t b = ((uint32_t)h) << 16;
    float f;
    memcpy(&f, &b, 4);
    return f;
}

static uint16_t bf16_store(float f) {
    uint32_t b;
    memcpy(&b, &f, 4);
    if ((b & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((b >> 16) | 0x40u); /* quiet NaN */
    uint32_t lsb = (b >> 16) & 1u;
    return (uint16_t)((b + 0x7FFFu + lsb) >> 16); /* round to nearest, ties to even */
}

/* --------------------------------------------------------- Jacobi-1D --- */

#define JACOBI1D_BODY(T_, THREE)                                              \
    T_* A = (T_*)malloc(sizeof(T_) * n);                                      \
    T_* B = (T_*)malloc(sizeof(T_) * n);                                      \
    if (!A || !B) { free(A); free(B); return -1; }                            \
    memcpy(A, in, sizeof(T_) * n);                                            \
    memcpy(B, in, sizeof(T_) * n);                                            \
    for (int64_t t = 0; t < T; ++t) {                                         \
        for (int64_t i = 1; i < n - 1; ++i)                                   \
            B[i] = ((A[i - 1] + A[i]) + A[i + 1]) / THREE;                    \
        T_* tmp = A; A = B; B = tmp;                                          \
    }                                                                         \
    memcpy(out, A, sizeof(T_) * n);                                           \
    free(A); free(B);                                                         \
    return 0;

int oracle_jacobi1d_f64(const double* in, double* out, int64_t n, int64_t T) {
    JACOBI1D_BODY(double, 3.0)
}

int oracle_jacobi1d_f32(const float* in, float* out, int64_t n, int64_t T) {
    JACOBI1D_BODY(float, 3.0f)
}

int oracle_jacobi1d_bf16(const uint16_t* in, uint16_t* out, int64_t n, int64_t T) {
    uint16_t* A = (uint16_t*)malloc(2 * n);
    uint16_t* B = (uint16_t*)malloc(2 * n);
    if (!A || !B) { free(A); free(B); return -1; }
    memcpy(A, in, 2 * n);
    memcpy(B, in, 2 * n);
    for (int64_t t = 0; t < T; ++t) {
        for (int64_t i = 1; i < n - 1; ++i) {
            float l = bf16_load(A[i - 1]), c = bf16_load(A[i]), r = bf16_load(A[i + 1]);
            B[i] = bf16_store(((l + c) + r) / 3.0f);
        }
        uint16_t* tmp = A; A = B; B = tmp;
    }
    memcpy(out, A, 2 * n);
    free(A); free(B);
    return 0;
}

/* --------------------------------------------------------- Jacobi-2D --- */

#define JACOBI2D_BODY(T_, FIFTH)                                              \
    const int64_t sz = ny * nx;                                               \
    T_* A = (T_*)malloc(sizeof(T_) * sz);                                     \
    T_* B = (T_*)malloc(sizeof(T_) * sz);                                     \
    if (!A || !B) { free(A); free(B); return -1; }                            \
    memcpy(A, in, sizeof(T_) * sz);                                           \
    memcpy(B, in, sizeof(T_) * sz);                                           \
    for (int64_t t = 0; t < T; ++t) {                                         \
        _Pragma("omp parallel for schedule(static)")                          \
        for (int64_t y = 1; y < ny - 1; ++y) {                                \
            for (int64_t x = 1; x < nx - 1; ++x) {                            \
                T_ c = A[y * nx + x];                                         \
                T_ n_ = A[(y - 1) * nx + x];                                  \
                T_ s = A[(y + 1) * nx + x];                                   \
                T_ e = A[y * nx + x + 1];                                     \
                T_ w = A[y * nx + x - 1];                                     \
                B[y * nx + x] = FIFTH * ((((c + n_) + s) + e) + w);           \
            }                                                                 \
        }                                                                     \
        T_* tmp = A; A = B; B = tmp;                                          \
    }                                                                         \
    memcpy(out, A, sizeof(T_) * sz);                                          \
    free(A); free(B);                                                         \
    return 0;

int oracle_jacobi2d_f64(const double* in, double* out, int64_t ny, int64_t nx, int64_t T) {
    JACOBI2D_BODY(double, 0.2)
}

int oracle_jacobi2d_f32(const float* in, float* out, int64_t ny, int64_t nx, int64_t T) {
    JACOBI2D_BODY(float, 0.2f)
}

int oracle_jacobi2d_bf16(const uint16_t* in, uint16_t* out, int64_t ny, int64_t nx, int64_t T) {
    const int64_t sz = ny * nx;
    uint16_t* A = (uint16_t*)malloc(2 * sz);
    uint16_t* B = (uint16_t*)malloc(2 * sz);
    if (!A || !B) { free(A); free(B); return -1; }
    memcpy(A, in, 2 * sz);
    memcpy(B, in, 2 * sz);
    for (int64_t t = 0; t < T; ++t) {
#pragma omp parallel for schedule(static)
        for (int64_t y = 1; y < ny - 1; ++y) {
            for (int64_t x = 1; x < nx - 1; ++x) {
                float c = bf16_load(A[y * nx + x]);
                float n_ = bf16_load(A[(y - 1) * nx + x]);
                float s = bf16_load(A[(y + 1) * nx + x]);
                float e = bf16_load(A[y * nx + x + 1]);
                float w = bf16_load(A[y * nx + x - 1]);
                B[y * nx + x] = bf16_store(0.2f * ((((c + n_) + s) + e) + w));
            }
        }
        uint16_t* tmp = A; A = B; B = tmp;
    }
    memcpy(out, A, 2 * sz);
    free(A); free(B);
    return 0;
}

/* ----------------------------------------------------------- Heat-3D --- */

#define HEAT3D_BODY(T_, TWO, EIGHTH)                                          \
    const int64_t sz = nz * ny * nx, py = nx, pz = ny * nx;                   \
    T_* A = (T_*)malloc(sizeof(T_) * sz);                                     \
    T_* B = (T_*)malloc(sizeof(T_) * sz);                                     \
    if (!A || !B) { free(A); free(B); return -1; }                            \
    memcpy(A, in, sizeof(T_) * sz);                                           \
    memcpy(B, in, sizeof(T_) * sz);                                           \
    for (int64_t t = 0; t < T; ++t) {                                         \
        _Pragma("omp parallel for schedule(static)")                          \
        for (int64_t z = 1; z < nz - 1; ++z) {                                \
            for (int64_t y = 1; y < ny - 1; ++y) {                            \
                for (int64_t x = 1; x < nx - 1; ++x) {                        \
                    int64_t p = z * pz + y * py + x;                          \
                    T_ u = A[p];                                              \
                    T_ dx = (A[p + 1] - TWO * u) + A[p - 1];                  \
                    T_ dy = (A[p + py] - TWO * u) + A[p - py];                \
                    T_ dz = (A[p + pz] - TWO * u) + A[p - pz];                \
                    B[p] = u + EIGHTH * ((dx + dy) + dz);                     \
                }                                                             \
            }                                                                 \
        }                                                                     \
        T_* tmp = A; A = B; B = tmp;                                          \
    }                                                                         \
    memcpy(out, A, sizeof(T_) * sz);                                          \
    free(A); free(B);                                                         \
    return 0;

int oracle_heat3d_f64(const double* in, double* out, int64_t nz, int64_t ny, int64_t nx, int64_t T) {
    HEAT3D_BODY(double, 2.0, 0.125)
}

int oracle_heat3d_f32(const float* in, float* out, int64_t nz, int64_t ny, int64_t nx, int64_t T) {
    HEAT3D_BODY(float, 2.0f, 0.125f)
}

int oracle_heat3d_bf16(const uint16_t* in, uint16_t* out, int64_t nz, int64_t ny, int64_t nx, int64_t T) {
    const int64_t sz = nz * ny * nx, py = nx, pz = ny * nx;
    uint16_t* A = (uint16_t*)malloc(2 * sz);
    uint16_t* B = (uint16_t*)malloc(2 * sz);
    if (!A || !B) { free(A); free(B); return -1; }
    memcpy(A, in, 2 * sz);
    memcpy(B, in, 2 * sz);
    for (int64_t t = 0; t < T; ++t) {
#pragma omp parallel for schedule(static)
        for (int64_t z = 1; z < nz - 1; ++z) {
            for (int64_t y = 1; y < ny - 1; ++y) {
                for (int64_t x = 1; x < nx - 1; ++x) {
                    int64_t p = z * pz + y * py + x;
                    float u = bf16_load(A[p]);
                    float dx = (bf16_load(A[p + 1]) - 2.0f * u) + bf16_load(A[p - 1]);
                    float dy = (bf16_load(A[p + py]) - 2.0f * u) + bf16_load(A[p - py]);
                    float dz = (bf16_load(A[p + pz]) - 2.0f * u) + bf16_load(A[p - pz]);
                    B[p] = bf16_store(u + 0.125f * ((dx + dy) + dz));
                }
            }
        }
        uint16_t* tmp = A; A = B; B = tmp;
    }
    memcpy(out, A, 2 * sz);
    free(A); free(B);
    return 0;
}

/* ------------------------------------------- sampled single outputs --- */
/*
 * Value of one output point u_T[y][x] (Jacobi-2D, f64) from its domain of
 * dependence only: u_s at distance d (Chebyshev) from (y, x) is needed only
 * while d <= T - s, so step s updates the interior points of that square.
 * Same update rule and order as the full oracle, hence the same bits.
 */
double oracle_jacobi2d_point_f64(const double* in, int64_t ny, int64_t nx, int64_t T,
                                 int64_t y, int64_t x) {
    const int64_t r = T + 1;
    const int64_t y0 = y - r < 0 ? 0 : y - r, y1 = y + r > ny - 1 ? ny - 1 : y + r;
    const int64_t x0 = x - r < 0 ? 0 : x - r, x1 = x + r > nx - 1 ? nx - 1 : x + r;
    const int64_t wy = y1 - y0 + 1, wx = x1 - x0 + 1;
    double* A = (double*)malloc(sizeof(double) * wy * wx);
    double* B = (double*)malloc(sizeof(double) * wy * wx);
    if (!A || !B) { free(A); free(B); return NAN; }
    for (int64_t i = 0; i < wy; ++i)
        for (int64_t j = 0; j < wx; ++j) A[i * wx + j] = B[i * wx + j] = in[(y0 + i) * nx + x0 + j];
    for (int64_t s = 1; s <= T; ++s) {
        const int64_t d = T - s;
        for (int64_t yy = y - d; yy <= y + d; ++yy) {
            if (yy < 1 || yy > ny - 2) continue;
            for (int64_t xx = x - d; xx <= x + d; ++xx) {
                if (xx < 1 || xx > nx - 2) continue;
                const int64_t i = yy - y0, j = xx - x0;
                double c = A[i * wx + j];
                double n_ = A[(i - 1) * wx + j];
                double so = A[(i + 1) * wx + j];
                double e = A[i * wx + j + 1];
                double w = A[i * wx + j - 1];
                B[i * wx + j] = 0.2 * ((((c + n_) + so) + e) + w);
            }
        }
        double* tmp = A; A = B; B = tmp;
    }
    double v = A[(y - y0) * wx + (x - x0)];
    free(A); free(B);
    return v;
}

/* ------------------------------------------------------ matrix chain --- */
/*
 * p: N+1 dimensions (matrix A_i is p[i-1] x p[i], i = 1..N).
 * C: N*N row-major, C[(i-1)*N + (j-1)] holds the cost of A_i..A_j for i <= j;
 *    the lower triangle is set to 0.
 * split (nullable): same layout, the smallest optimal k (i <= k < j), 0 on
 *    the diagonal.
 * A transposed mirror CT[j][k] = C[k][j] keeps the inner loop unit-stride; it
 * is a layout choice, not a reordering.
 */
int oracle_matrix_chain(const int64_t* p, int64_t N, int64_t* C, int64_t* split) {
    if (N < 1) return -1;
    int64_t* CT = (int64_t*)calloc((size_t)N * N, sizeof(int64_t));
    if (!CT) return -1;
    memset(C, 0, sizeof(int64_t) * N * N);
    if (split) memset(split, 0, sizeof(int64_t) * N * N);
    /* 0-based: cell (a, b) with a <= b is A_{a+1}..A_{b+1}; its weight for
       split point k (a <= k < b) is p[a] * p[k+1] * p[b+1]. */
    for (int64_t len = 2; len <= N; ++len) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t a = 0; a <= N - len; ++a) {
            const int64_t b = a + len - 1;
            int64_t best = INT64_MAX, arg = a;
            const int64_t* row = C + a * N;    /* C[a][k]   */
            const int64_t* col = CT + b * N;   /* C[k+1][b] */
            for (int64_t k = a; k < b; ++k) {
                int64_t q = row[k] + col[k + 1] + p[a] * p[k + 1] * p[b + 1];
                if (q < best) { best = q; arg = k; }
            }
            C[a * N + b] = best;
            CT[b * N + a] = best;
            if (split) split[a * N + b] = arg + 1; /* 1-based k of A_k | A_{k+1} */
        }
    }
    free(CT);
    return 0;
}

/* ---------------------------------------------------- Gauss-Seidel-2D --- */
/* In-place Gauss-Seidel sweeps of the 5-point average over the interior, in
 * lexicographic order (rows outer, columns inner): each point is replaced
 * by 0.2*((((c + n) + s) + e) + w) where n and w already hold this sweep's
 * values and c, s, e the previous sweep's.  The dependence inside a time
 * step is what separates it from Jacobi (Section 6.2 discussion of
 * Gauss-Seidel style stencils; Table 2, GS-2D). */
int oracle_gs2d_f64(const double* in, double* out, int64_t ny, int64_t nx, int64_t T) {
    memcpy(out, in, sizeof(double) * ny * nx);
    for (int64_t t = 0; t < T; ++t)
        for (int64_t y = 1; y < ny - 1; ++y)
            for (int64_t x = 1; x < nx - 1; ++x) {
                double* u = out + y * nx + x;
                *u = 0.2 * ((((u[0] + u[-nx]) + u[nx]) + u[1]) + u[-1]);
            }
    return 0;
}

/* ---------------------------------------------------------- FDTD-2D --- */
/* Three-statement time loop (an imperfect nest: three loop nests inside the
 * time loop; Section 4.4, Table 2 FDTD-2D), the 2D transverse-electric Yee
 * scheme on fields ex, ey, hz of ny x nx cells, updated in place:
 *   ey[i][j] -= CE * (hz[i][j] - hz[i-1][j])                     1 <= i < ny,  0 <= j < nx
 *   ex[i][j] += CE * (hz[i][j] - hz[i][j-1])                     0 <= i < ny,  1 <= j < nx
 *   hz[i][j] -= CH * ((ey[i+1][j] - ey[i][j]) - (ex[i][j+1] - ex[i][j]))
 *                                                                0 <= i < ny-1, 0 <= j < nx-1
 * Cells outside those ranges keep their values (fixed edges). */
#define FDTD_CE 0.25
#define FDTD_CH 0.5
int oracle_fdtd2d_f64(double* ex, double* ey, double* hz, int64_t ny, int64_t nx, int64_t T) {
    for (int64_t t = 0; t < T; ++t) {
        for (int64_t i = 1; i < ny; ++i)
            for (int64_t j = 0; j < nx; ++j)
                ey[i * nx + j] = ey[i * nx + j] - FDTD_CE * (hz[i * nx + j] - hz[(i - 1) * nx + j]);
        for (int64_t i = 0; i < ny; ++i)
            for (int64_t j = 1; j < nx; ++j)
                ex[i * nx + j] = ex[i * nx + j] + FDTD_CE * (hz[i * nx + j] - hz[i * nx + j - 1]);
        for (int64_t i = 0; i < ny - 1; ++i)
            for (int64_t j = 0; j < nx - 1; ++j)
                hz[i * nx + j] = hz[i * nx + j] - FDTD_CH * ((ey[(i + 1) * nx + j] - ey[i * nx + j]) -
                                                             (ex[i * nx + j + 1] - ex[i * nx + j]));
    }
    return 0;
}

/* ------------------------------------------------ motivating example --- */
/* The appendix's motivating 1D program (Memory Allocation, Fig. motiv), with
 * the two-buffer allocation X[t mod 2][i] of the original code:
 *   X[0][i] = A[i];
 *   for t = 1..T: for i = 1..N-2:  X[t%2][i] = f(X[(t-1)%2][i-1], X[(t-1)%2][i],
 *                                                X[(t-1)%2][i+1], X[(t-1)%2][0])   (S1)
 *                 X[t%2][0] = g(X[(t-1)%2][0]);  X[t%2][N-1] = g(X[(t-1)%2][N-1])  (S2, S3)
 *   out[i] = X[T%2][i].
 * The paper leaves f and g abstract; here
 *   f(a, b, c, d) = 0.25 * (((a + b) + c) + d),   g(y) = 0.5 * y + 0.25. */
static inline double motiv_f(double a, double b, double c, double d) { return 0.25 * (((a + b) + c) + d); }
static inline double motiv_g(double y) { return 0.5 * y + 0.25; }

int oracle_motiv_f64(const double* A, double* out, int64_t N, int64_t T) {
    double* X = (double*)malloc(sizeof(double) * 2 * N);
    if (!X) return -1;
    memcpy(X, A, sizeof(double) * N);
    memcpy(X + N, A, sizeof(double) * N);
    for (int64_t t = 1; t <= T; ++t) {
        double* cur = X + (t % 2) * N;
        const double* old = X + ((t - 1) % 2) * N;
        for (int64_t i = 1; i < N - 1; ++i) cur[i] = motiv_f(old[i - 1], old[i], old[i + 1], old[0]);
        cur[0] = motiv_g(old[0]);
        cur[N - 1] = motiv_g(old[N - 1]);
    }
    memcpy(out, X + (T % 2) * N, sizeof(double) * N);
    free(X);
    return 0;
}
