// Interval DP (matrix chain / optimal parenthesization) on b x b tiles of the
// upper triangle of C:
//   C[i][i] = 0,  C[i][j] = min_{i<=k<j} C[i][k] + C[k+1][j] + p[i-1] p[k] p[j]
// (0-based cells here: cell (a, c) covers A_{a+1}..A_{c+1}; its weight for
// split k' in [a, c) is p[a] * p[k'+1] * p[c+1]).
//
// The reduction over k is reordered freely (the Guibas-Kung-Thompson
// reordering that makes all three dimensions of the OSP nest tileable,
// Section 5.1.2): integer min and + are exact, so every order and every split
// of the k range gives the same bits.  For tile (I, J), a split k belongs to
//   * the external range [(I+1)b-1, Jb-1]: both operands lie in tiles that a
//     previous phase finished -> min-plus product of complete tiles
//     (k_ext), split over blocks, combined with atomicMin;
//   * the internal ranges [i, (I+1)b-2] and [Jb, j-1]: one operand lies in
//     tile (I, J) itself, below or left of the cell -> k_fin processes the
//     tile's cells by anti-diagonals after the external part is complete.
// A diagonal tile (I, I) has only internal splits.
//
// 32-bit path: exact while (N-1) * pmax^3 < 2^32, since every candidate is at
// most (j-i) * pmax^3; the weight is p[a]*p[c+1] (< 2^24) times p[k'+1]
// (< 2^24), one v_mad_u32_u24.  64-bit path otherwise.
#include "common.hpp"
#include "kernels.hpp"

namespace pcot {

enum : int { DP_INIT = 0, DP_ITEMS = 1, DP_FINISH = 2 };

struct DPLaunch {
    const long long* p;  // N+1 dimensions (device)
    void* Cw;            // working matrix, N x N, u32 or i64 (device)
    long long* C;        // output, Nout x Nout int64 (device)
    int N, Nout, b;      // N: padded to a multiple of b (dims past Nout are 1)
    const int2* tiles;   // (I, J) of the phase (device)
    int ntiles;
    const int4* items;   // external work items: ((I << 16) | J, k_begin, k_end, 0)
    int nitems;
    unsigned* hdr;
    long long pmax;
};

namespace {

template <typename V> struct DV;
template <> struct DV<unsigned> {
    static constexpr unsigned INF = 0xFFFFFFFFu;
    static __device__ __forceinline__ unsigned madw(unsigned w, unsigned pk, unsigned a) {
        return __umul24(w, pk) + a;  // w, pk < 2^24: one v_mad_u32_u24
    }
    static __device__ __forceinline__ unsigned add(unsigned a, unsigned b) { return a + b; }
    static __device__ __forceinline__ void amin(unsigned* p, unsigned v) { atomicMin(p, v); }
};
template <> struct DV<long long> {
    static constexpr long long INF = 0x7FFFFFFFFFFFFFFFLL;
    // wrapping arithmetic: exact for every candidate that can win (they are
    // below 2^62); discarded slots may hold INF operands
    static __device__ __forceinline__ long long madw(long long w, long long pk, long long a) {
        return (long long)((unsigned long long)w * (unsigned long long)pk + (unsigned long long)a);
    }
    static __device__ __forceinline__ long long add(long long a, long long b) {
        return (long long)((unsigned long long)a + (unsigned long long)b);
    }
    static __device__ __forceinline__ void amin(long long* p, long long v) { atomicMin(p, v); }
};

// ---------------------------------------------------------------- setup ---
// p' = p[0..Nout], then 1 up to index N (padding matrices of 1 x 1 at the end
// of the chain: a cell (i, j) only reads splits k < j, so real cells never
// see them).
__global__ void k_dp_pad(const long long* p, long long* pp, int Nout, int N) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= N; i += gridDim.x * blockDim.x)
        pp[i] = i <= Nout ? p[i] : 1;
}

// Cw: off-diagonal upper cells INF, diagonal 0; C: 0 everywhere (the lower
// triangle stays 0).  Checks 1 <= p <= pmax.
template <typename V>
__global__ void k_dp_init(DPLaunch a) {
    const size_t n = (size_t)a.N * a.N;
    V* Cw = (V*)a.Cw;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / a.N), c = (int)(e % a.N);
        Cw[e] = r < c ? DV<V>::INF : (V)0;
        if (r < a.Nout && c < a.Nout) a.C[(size_t)r * a.Nout + c] = 0;
    }
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= a.N; i += gridDim.x * blockDim.x) {
        const long long v = a.p[i];
        if (i <= a.Nout && (v < 1 || v > a.pmax))
            __hip_atomic_store(a.hdr + HDR_ERROR, DEVERR_INPUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ------------------------------------------------------- external part ---
// One block per work item: a B x B output tile, k in [k0, k1).  Each thread
// owns an R x R micro-tile; operand tiles go through LDS in KT-deep slices
// (A transposed so a thread's R rows are contiguous).  Every load of a slice
// is issued before its LDS stores, so a slice costs one memory round trip,
// and a slice takes a whole k-chunk of up to 64 splits (16 for B = 64, where
// the finishing pass that shares the kernel leaves less LDS); the A panel is
// read along its rows (consecutive k), the B panel along its rows
// (consecutive j).
// NT threads per block, each owning one micro-tile ((B/R)^2 == NT).
template <typename V, int B, int R, int NT>
__device__ __forceinline__ void dp_ext_item(const DPLaunch& a, int item) {
    constexpr int KT = B <= 32 ? 64 : 16;
    constexpr int PER = KT * B / NT;  // values per thread and panel in a slice
    constexpr int TPR = B / R;        // threads per row of micro-tiles
    static_assert(TPR * TPR == NT, "micro-tile layout");
    static_assert(PER >= 1 && PER * NT == KT * B && NT >= KT, "staging layout");
    __shared__ V As[KT][B + 1];  // As[kk][r] = C[I*B + r][k0 + kk]
    __shared__ V Bs[KT][B];      // Bs[kk][c] = C[k0 + kk + 1][J*B + c]
    __shared__ V Ps[KT];         // p[k + 1]
    const int4 it = a.items[item];
    const int I = it.x >> 16, J = it.x & 0xFFFF;  // target tile (I, J)
    const int N = a.N;
    const V* Cw = (const V*)a.Cw;
    const int tid = threadIdx.x;
    const int tr = tid / TPR, tc = tid % TPR;  // micro-tile coordinates
    const int row0 = I * B + tr * R, col0 = J * B + tc * R;
    V w[R][R], m[R][R];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < R; ++c) {
            w[r][c] = (V)a.p[row0 + r] * (V)a.p[col0 + c + 1];
            m[r][c] = DV<V>::INF;
        }
    for (int k0 = it.y; k0 < it.z; k0 += KT) {
        // past the end of the range: a candidate of INF, which never wins
        V ra[PER], rb[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + u * NT;
            const int ka = e % KT, xa = e / KT, kb = e / B, xb = e % B;
            ra[u] = k0 + ka < it.z ? Cw[(size_t)(I * B + xa) * N + k0 + ka] : DV<V>::INF;
            rb[u] = k0 + kb < it.z ? Cw[(size_t)(k0 + kb + 1) * N + J * B + xb] : (V)0;
        }
        const V rp = (tid < KT && k0 + tid < it.z) ? (V)a.p[k0 + tid + 1] : (V)0;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + u * NT;
            As[e % KT][e / KT] = ra[u];
            Bs[e / B][e % B] = rb[u];
        }
        if (tid < KT) Ps[tid] = rp;
        __syncthreads();
        // the slice's rows in use, rounded up to the unroll (rows past the
        // range hold INF / 0); the same for the whole block
        const int kn = (min(KT, it.z - k0) + 3) & ~3;
        {
#pragma unroll 4
            for (int kk = 0; kk < kn; ++kk) {
                V av[R], bv[R];
#pragma unroll
                for (int r = 0; r < R; ++r) av[r] = As[kk][tr * R + r];
#pragma unroll
                for (int c = 0; c < R; ++c) bv[c] = Bs[kk][tc * R + c];
                const V pk = Ps[kk];
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int c = 0; c < R; ++c) {
                        const V qv = DV<V>::madw(w[r][c], pk, av[r]) + bv[c];
                        m[r][c] = qv < m[r][c] ? qv : m[r][c];
                    }
            }
        }
        __syncthreads();
    }
    V* Cm = (V*)a.Cw;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < R; ++c) DV<V>::amin(Cm + (size_t)(row0 + r) * N + col0 + c, m[r][c]);
}

// Minimum over groups of TPC adjacent lanes (TPC in {2, ..., 32}) with DPP
// lane moves: swap neighbours, swap pairs within a quad, mirror the two quads
// of each half row (lane i of the 8 meets lane 7-i), mirror the row of 16;
// every lane of a row then holds the row's minimum.  A group of 32 (two rows)
// ends with a broadcast of lane 15 of each even row into the odd row after
// it, so the group's last lane (in the odd row) holds the minimum.  Only the
// group's last lane's result is defined.
__device__ __forceinline__ unsigned dpp_move(unsigned v, int ctrl) {
    switch (ctrl) {
        case 0: return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
        case 1: return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
        case 2: return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
        case 3: return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);  // row_mirror
        // row_bcast:15 into rows 1 and 3; rows 0 and 2 keep their own value
        default: return (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x142, 0xA, 0xF, false);
    }
}
__device__ __forceinline__ long long dpp_move(long long v, int ctrl) {
    const unsigned lo = dpp_move((unsigned)(unsigned long long)v, ctrl);
    const unsigned hi = dpp_move((unsigned)((unsigned long long)v >> 32), ctrl);
    return (long long)(((unsigned long long)hi << 32) | lo);
}
template <int TPC, typename V>
__device__ __forceinline__ V group_min(V v) {
    static_assert(TPC == 2 || TPC == 4 || TPC == 8 || TPC == 16 || TPC == 32, "group of 2 to 32 lanes");
#pragma unroll
    for (int c = 0; (1 << c) < TPC; ++c) {
        const V o = dpp_move(v, c);
        v = o < v ? o : v;
    }
    return v;
}

// -------------------------------------------------------- finishing part ---
// One block (WAVE: one wave) per tile.  Cells are taken by anti-diagonals of
// (u, v) = ((I+1)B-1-i, j-JB): a cell's internal operands lie below it (same
// column) or left of it (same row), i.e. on earlier anti-diagonals.  Each cell
// is handled by TPC threads that split its internal k range, then
// min-reduce.  With one wave the anti-diagonals need no block barrier: the
// LDS accesses of a wave are carried out in the order it issues them, so a
// wave barrier (which only keeps the compiler from moving them) orders the
// steps.
template <typename V, int B, int NT, bool WAVE = false>
__device__ __forceinline__ void dp_fin_tile(const DPLaunch& a, int tile) {
    static_assert(!WAVE || NT == 64, "one wave");
    auto sync = [] {
        if constexpr (WAVE) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            __syncthreads();
        }
    };
    constexpr int TPC = NT / B;    // threads per cell
    constexpr int WS = 2 * B + 1;  // row stride of W
    constexpr int SS = B + 1;      // row stride of S
    // A cell's in-tile splits, indexed x: x in [li, kA1) are the splits k of
    // block I (local k = x), x in [B, B + lj) those of block J (local k =
    // x - B).  Both parts read their operands from one array each:
    //   W[r][x]  row operand C[i][k]:    x < B tile (I, I) (the tile itself
    //            when diagonal), x >= B the tile (I, J);
    //   S[y][c]  column operand C[k+1][j], y = x + 1: y < B the tile (I, J),
    //            y > B tile (J, J);
    //   PC[y]    p[k+1]: y <= B p[I*B + y], y > B p[J*B + y - B].
    // The tile is held twice (in W's right half, or left half when diagonal,
    // and in S's upper half) and every cell is written to both.
    __shared__ V W[B * WS];
    __shared__ V S[2 * B * SS];
    __shared__ V PC[2 * B + 1];
    const int2 tj = a.tiles[tile];
    const int I = tj.x, J = tj.y;
    const int N = a.N;
    V* Cw = (V*)a.Cw;
    const int tid = threadIdx.x;
    const bool diag = I == J;
    const int wt = diag ? 0 : B;  // the tile's column offset in W
    for (int e = tid; e < B * B; e += NT) {
        const int r = e / B, c = e % B;
        const V t = Cw[(size_t)(I * B + r) * N + J * B + c];
        W[r * WS + wt + c] = t;
        S[r * SS + c] = t;
        if (!diag) {
            W[r * WS + c] = Cw[(size_t)(I * B + r) * N + I * B + c];
            S[(B + r) * SS + c] = Cw[(size_t)(J * B + r) * N + J * B + c];
        }
    }
    for (int y = tid; y <= 2 * B; y += NT) PC[y] = (V)a.p[y <= B ? I * B + y : J * B + y - B];
    sync();
    const int cell = tid / TPC, part = tid % TPC;
    for (int s = 0; s <= 2 * B - 2; ++s) {
        // cell index along the anti-diagonal: u from max(0, s-B+1)
        const int u = (s < B ? 0 : s - B + 1) + cell;
        const int v = s - u;
        const bool act = u < B && v >= 0 && v < B && u <= s;
        V best = DV<V>::INF;
        int li = 0, lj = 0;
        bool live = false;
        if (act) {
            li = B - 1 - u;  // i = I*B + li
            lj = v;          // j = J*B + lj
            live = diag ? li < lj : true;
            if (live) {
                // every lane of the cell starts from the cell's external
                // minimum (INF on diagonal tiles), read with the operands so
                // that the step has one round of LDS reads; only this cell
                // writes it, at the end of this step
                best = S[li * SS + lj];
                const V w = PC[li] * PC[B + 1 + lj];  // p[i] * p[j+1]
                const int n1 = (diag ? lj : B - 1) - li, n = n1 + (diag ? 0 : lj);
                const int shiftA = li, shiftB = B - n1;
                const V* Wr = W + li * WS;
                // a fixed, unrolled number of slots per thread (at most 2B - 2
                // splits per cell), so that all LDS reads of a step are in
                // flight together; a slot past n reads a valid cell and is
                // discarded
#pragma unroll
                for (int it = 0; it < (2 * B + TPC - 1) / TPC; ++it) {
                    const int q = part + it * TPC;
                    const int x = min(q + (q < n1 ? shiftA : shiftB), 2 * B - 2);
                    const V cand = DV<V>::add(DV<V>::madw(w, PC[x + 1], Wr[x]), S[(x + 1) * SS + lj]);
                    best = (q < n && cand < best) ? cand : best;
                }
            }
        }
        // min over the cell's TPC threads (adjacent lanes of one wave), held
        // by the group's last lane
        best = group_min<TPC>(best);
        if (act && part == TPC - 1 && live) {
            S[li * SS + lj] = best;
            W[li * WS + wt + lj] = best;
        }
        sync();
    }
    for (int e = tid; e < B * B; e += NT) {
        const int r = e / B, c = e % B;
        const int gi = I * B + r, gj = J * B + c;
        if (gi <= gj) {
            const V v = S[r * SS + c];
            Cw[(size_t)gi * N + gj] = v;
            if (gj < a.Nout) a.C[(size_t)gi * a.Nout + gj] = (long long)v;
        }
    }
}

// External items alone (they need the tiles finished by the previous launch).
template <typename V, int B, int R>
__global__ void __launch_bounds__(256) k_dp_ext(DPLaunch a) {
    dp_ext_item<V, B, R, 256>(a, blockIdx.x);
}

// A phase's finishing pass together with the external items of the next
// phase whose operand tiles were finished before this launch: blocks
// [0, ntiles) finish tiles, the rest take items.  The two sets touch
// disjoint tiles (items only read finished tiles and atomically lower cells
// of next-phase tiles).
// 1024 threads: a cell of the finishing pass gets 1024 / B lanes (b = 32, 64).
template <typename V, int B, int R>
__global__ void __launch_bounds__(1024) k_dp_fin(DPLaunch a) {
    // a cell gets at most 32 lanes (the group minimum stays inside a half wave)
    constexpr int FT = B * 32 < 1024 ? B * 32 : 1024;
    if ((int)blockIdx.x < a.ntiles)
        dp_fin_tile<V, B, FT>(a, blockIdx.x);
    else
        dp_ext_item<V, B, B / 32, 1024>(a, blockIdx.x - a.ntiles);
}

// b = 16: the finishing pass of a tile is one wave (4 lanes per cell), in
// 256-thread blocks shared with the external items (at N = 4096 1.56x the
// 1024-thread pass; at b = 32 two lanes per cell walk 32 splits each and the
// block pass stays 3.4x faster).
template <typename V, int B, int R>
__global__ void __launch_bounds__(256) k_dp_finw(DPLaunch a) {
    if ((int)blockIdx.x < a.ntiles) {
        if (threadIdx.x < 64) dp_fin_tile<V, B, 64, true>(a, blockIdx.x);
    } else {
        dp_ext_item<V, B, R, 256>(a, blockIdx.x - a.ntiles);
    }
}

template <typename V, int B>
hipError_t launch_phase_t(const DPLaunch& a, int mode, hipStream_t s) {
    if (mode == DP_INIT) {
        hipLaunchKernelGGL((k_dp_init<V>), dim3(2048), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    constexpr int R = B == 16 ? 1 : (B == 32 ? 2 : (B == 64 ? 4 : 8));
    if (mode == DP_ITEMS) {
        if (a.nitems > 0) hipLaunchKernelGGL((k_dp_ext<V, B, R>), dim3(a.nitems), dim3(256), 0, s, a);
    } else if (a.ntiles + a.nitems > 0) {
        if constexpr (B == 16)
            hipLaunchKernelGGL((k_dp_finw<V, B, R>), dim3(a.ntiles + a.nitems), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_dp_fin<V, B, R>), dim3(a.ntiles + a.nitems), dim3(1024), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace

bool dp_block_supported(int b) { return b == 16 || b == 32 || b == 64; }

hipError_t launch_dp_pad(const long long* p, long long* pp, int Nout, int N, hipStream_t s) {
    hipLaunchKernelGGL(k_dp_pad, dim3((N + 256) / 256), dim3(256), 0, s, p, pp, Nout, N);
    return hipGetLastError();
}

// One launch of a DP plan: the initialisation of the working matrices, a set
// of external items, or a finishing pass with the items that run beside it.
hipError_t launch_dp_phase(bool wide, const DPLaunch& a, int mode, hipStream_t s) {
    if (!wide) {
        if (a.b == 16) return launch_phase_t<unsigned, 16>(a, mode, s);
        if (a.b == 32) return launch_phase_t<unsigned, 32>(a, mode, s);
        return launch_phase_t<unsigned, 64>(a, mode, s);
    }
    if (a.b == 16) return launch_phase_t<long long, 16>(a, mode, s);
    if (a.b == 32) return launch_phase_t<long long, 32>(a, mode, s);
    return launch_phase_t<long long, 64>(a, mode, s);
}

}  // namespace pcot
