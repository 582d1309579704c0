// Time-skewed tile executor for the 5-point Jacobi-2D stencil.  Blocks take
// tiles from a device queue in schedule order and wait on per-tile
// dependency counters.
//
// A leaf (paper: the base function, Section 4.2) is the box
//   t in [t0, t0+nt) x jy in [jy0, jy0+by) x jx in [jx0, jx0+bx)
// of the skewed space jy = y + t, jx = x + t.  Level t at (jy, jx) updates
// u_{t+1}[jy-t][jx-t] from level t-1 outputs at
//   c (jy-1, jx-1), n (jy-2, jx-1), s (jy, jx-1), e (jy-1, jx), w (jy-1, jx-2),
// so inside a tile every input comes from the same or a lower row and column.
//
// Mapping onto CDNA:
//  * lanes own columns: lane l holds jx = jx0 + l*C .. + C-1 (bx = 64*C);
//    the one- and two-column shifts cross lanes with DPP wave_shr:1;
//  * the block streams along jy; wave g of G owns levels [g*L, g*L+L) and
//    runs one row behind wave g-1, taking its input row from an LDS handoff
//    (one barrier per row), so a tile holds bt = G*L levels in registers and
//    each point crosses HBM once per tile instead of once per step;
//  * per level, the two previous input rows live in registers;
//  * inputs written by other tiles (the bottom plane u_t0, and the two-wide
//    low faces of every level) are read from the two t-mod-2 field buffers,
//    where the producing tiles left them; a tile writes its top plane and its
//    two-wide high faces at every level.
// Points outside the interior are carried through unchanged (identity), which
// reproduces the fixed boundary; outside-array positions never feed an
// interior point.  Tiles that lie entirely inside the interior take a path
// without any masking or clamping.
#include "common.hpp"
#include "kernels.hpp"

namespace pcot {

namespace {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Buffer selection by bit masks: a conditional pick between two struct
// fields would be lowered to an indexed load from a stack copy.
__device__ __forceinline__ uintptr_t pick(uintptr_t a, uintptr_t b, int sel_b) {
    const uintptr_t m = (uintptr_t)0 - (uintptr_t)(sel_b & 1);
    return (a & ~m) | (b & m);
}
template <typename S>
__device__ __forceinline__ const S* level_src(const TiledProblem& P, int t) {
    // buffer holding u_t
    const uintptr_t b = pick((uintptr_t)P.buf0, (uintptr_t)P.buf1, t);
    return (const S*)pick(b, (uintptr_t)P.in, t == 0);
}
template <typename S>
__device__ __forceinline__ S* level_dst(const TiledProblem& P, int t) {
    // buffer receiving u_{t+1} (the output of level t)
    return (S*)pick((uintptr_t)P.buf0, (uintptr_t)P.buf1, t + 1);
}

// v[0..N) = u[y][x .. x+N) with clamping to the array when BND.
template <typename S, bool BND, int N>
__device__ __forceinline__ void ldseg(const S* base, int ny, int nx, int y, int x,
                                      typename Tr<S>::A* v) {
    if (BND) y = clampi(y, 0, ny - 1);
    const S* row = base + (size_t)y * nx;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        int xx = x + i;
        if (BND) xx = clampi(xx, 0, nx - 1);
        v[i] = Tr<S>::ld(row + xx);
    }
}

__device__ __forceinline__ bool leaf_nonempty(const TiledProblem& P, int kt, int ky, int kx) {
    if (kt < 0 || ky < 0 || kx < 0 || kt >= P.cnt[0] || ky >= P.cnt[1] || kx >= P.cnt[2]) return false;
    const int tlo = kt * P.b[0];
    int tmin = tlo, tmax = min(tlo + P.b[0] - 1, P.T - 1);
    const int ylo = 1 + ky * P.b[1], xlo = 1 + kx * P.b[2];
    tmin = max(tmin, max(ylo - P.n[0] + 2, xlo - P.n[1] + 2));
    tmax = min(tmax, min(ylo + P.b[1] - 2, xlo + P.b[2] - 2));
    return tmin <= tmax;
}

__device__ __forceinline__ bool leaf_interior(const TiledProblem& P, int kt, int ky, int kx) {
    const int t0 = kt * P.b[0];
    const int nt = min(P.b[0], P.T - t0);
    const int t1 = t0 + nt - 1;
    const int jy0 = 1 + ky * P.b[1], jx0 = 1 + kx * P.b[2];
    return (jy0 - t1 >= 1) && (jy0 + P.b[1] - 1 - t0 <= P.n[0] - 2) && (jx0 - t1 >= 1) &&
           (jx0 + P.b[2] - 1 - t0 <= P.n[1] - 2);
}

template <typename S, int C, int L, int G, bool BND>
__device__ __forceinline__ void exec_tile(const TiledProblem& P, int kt, int ky, int kx,
                                          typename Tr<S>::A* hand, typename Tr<S>::A* lfs,
                                          typename Tr<S>::A* rfs) {
    using A = typename Tr<S>::A;
    constexpr int K = 64 / L;        // rows per staging chunk
    constexpr int ROW = 64 * C + 2;  // handoff row: 2 left-face values + 64*C columns
    const int lane = threadIdx.x & 63;
    const int w = uni((int)(threadIdx.x >> 6));
    const int ny = P.n[0], nx = P.n[1];
    const int bt = P.b[0], by = P.b[1], bx = 64 * C;
    const int t0 = kt * bt;
    const int nt = min(bt, P.T - t0);
    const int ttop = t0 + nt - 1;
    const int jy0 = 1 + ky * by, jx0 = 1 + kx * bx;
    const int tl0 = t0 + w * L;
    const int nl = clampi(nt - w * L, 0, L);
    const int jxl = jx0 + lane * C;
    A* mylfs = lfs + w * 128;
    A* myrfs = rfs + w * 128;

    A in1[L][C], in2[L][C], x1a[L], x1b[L], x2a[L];
    // ---- bottom faces: level t's input rows jy0-1 and jy0-2
#pragma unroll
    for (int l = 0; l < L; ++l) {
        if (l < nl) {
            const int t = tl0 + l;
            const S* src = level_src<S>(P, t);
            A seg[C + 2];
            ldseg<S, BND, C + 2>(src, ny, nx, jy0 - t, jxl - t - 1, seg);
            x1b[l] = seg[0];
            x1a[l] = seg[1];
#pragma unroll
            for (int c = 0; c < C; ++c) in1[l][c] = seg[2 + c];
            A seg2[C + 1];
            ldseg<S, BND, C + 1>(src, ny, nx, jy0 - t - 1, jxl - t, seg2);
            x2a[l] = seg2[0];
#pragma unroll
            for (int c = 0; c < C; ++c) in2[l][c] = seg2[1 + c];
        }
    }

    // ---- left faces (level t output at jx0-2, jx0-1), prefetched one chunk ahead:
    // lane i of the wave carries (row r0 + i / L, level i % L).
    A lfp0 = A(0), lfp1 = A(0);
    auto lf_fetch = [&](int r0) {
        const int rr = r0 + lane / L, l = lane % L, t = tl0 + l;
        if (rr < by && l < nl && t < ttop) {
            const S* src = (const S*)level_dst<S>(P, t);
            A v[2];
            ldseg<S, BND, 2>(src, ny, nx, jy0 + rr - t, jx0 - t - 2, v);
            lfp0 = v[0];
            lfp1 = v[1];
        }
    };
    // bottom plane (wave 0, level t0 input), prefetched one row ahead
    A bpn[C + 2];
    const S* bsrc = level_src<S>(P, t0);
    if (w == 0) ldseg<S, BND, C + 2>(bsrc, ny, nx, jy0 - t0 + 1, jxl - t0 - 1, bpn);
    if (nl > 0) lf_fetch(0);

    const int nsteps = by + G - 1;
    for (int S_ = 0; S_ < nsteps; ++S_) {
        const int r = S_ - w;
        if (nl > 0 && r >= 0 && r < by) {
            const int jy = jy0 + r;
            const int rk = r % K;
            if (rk == 0) {
                // publish this chunk's left faces to LDS, fetch the next chunk
                mylfs[2 * lane] = lfp0;
                mylfs[2 * lane + 1] = lfp1;
                __builtin_amdgcn_wave_barrier();
                lf_fetch(r + K);
            }
            // input row of this wave's first level
            A in0[C], x0a, x0b;
            if (w == 0) {
                x0b = bpn[0];
                x0a = bpn[1];
#pragma unroll
                for (int c = 0; c < C; ++c) in0[c] = bpn[2 + c];
                if (r + 1 < by) ldseg<S, BND, C + 2>(bsrc, ny, nx, jy + 1 - t0 + 1, jxl - t0 - 1, bpn);
            } else {
                const A* h = hand + ((w - 1) * 2 + ((S_ - 1) & 1)) * ROW;
                x0b = h[lane * C];
                x0a = h[lane * C + 1];
#pragma unroll
                for (int c = 0; c < C; ++c) in0[c] = h[2 + lane * C + c];
            }
#pragma unroll
            for (int l = 0; l < L; ++l) {
                if (l < nl) {
                    const int t = tl0 + l;
                    A out[C];
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        const A cc = c >= 1 ? in1[l][c - 1] : x1a[l];
                        const A nn = c >= 1 ? in2[l][c - 1] : x2a[l];
                        const A ss = c >= 1 ? in0[c - 1] : x0a;
                        const A ee = in1[l][c];
                        const A ww = c >= 2 ? in1[l][c - 2] : (c == 1 ? x1a[l] : x1b[l]);
                        A v = Tr<S>::rnd(jac2(cc, nn, ss, ee, ww));
                        if (BND) {
                            const int y = jy - t, x = jxl + c - t;
                            const bool inside = (y >= 1) & (y <= ny - 2) & (x >= 1) & (x <= nx - 2);
                            v = inside ? v : cc;
                        }
                        out[c] = v;
                    }
                    // rotate this level's input history
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        in2[l][c] = in1[l][c];
                        in1[l][c] = in0[c];
                    }
                    x2a[l] = x1a[l];
                    x1a[l] = x0a;
                    x1b[l] = x0b;

                    S* dst = level_dst<S>(P, t);
                    const int y = jy - t;
                    if (t == ttop || r >= by - 2) {
                        // top plane, or one of the two high rows of this level
                        S* row = dst + (size_t)(BND ? clampi(y, 0, ny - 1) : y) * nx;
#pragma unroll
                        for (int c = 0; c < C; ++c) {
                            const int x = jxl + c - t;
                            if (!BND || ((y >= 1) & (y <= ny - 2) & (x >= 1) & (x <= nx - 2)))
                                Tr<S>::st(row + x, out[c]);
                        }
                    }
                    if (t < ttop) {
                        const A lfA = mylfs[2 * (rk * L + l) + 1];  // column jx0-1
                        const A lfB = mylfs[2 * (rk * L + l)];      // column jx0-2
                        x0a = shr1(out[C - 1], lfA);
                        if constexpr (C >= 2) x0b = shr1(out[C - 2], lfB);
                        else x0b = shr1(x0a, lfB);
                        // stage the two-wide high face (columns jx0+bx-2, jx0+bx-1)
                        if (lane == 63) {
                            myrfs[2 * (rk * L + l)] = C >= 2 ? out[C >= 2 ? C - 2 : 0] : x0a;
                            myrfs[2 * (rk * L + l) + 1] = out[C - 1];
                        }
                        if (l == L - 1 && w < G - 1) {
                            A* h = hand + (w * 2 + (S_ & 1)) * ROW;
#pragma unroll
                            for (int c = 0; c < C; ++c) h[2 + lane * C + c] = out[c];
                            if (lane == 0) {
                                h[0] = lfB;
                                h[1] = lfA;
                            }
                        }
#pragma unroll
                        for (int c = 0; c < C; ++c) in0[c] = out[c];
                    }
                }
            }
            if (rk == K - 1 || r == by - 1) {
                // flush the staged high faces of this chunk: lane i -> (row, level)
                __builtin_amdgcn_wave_barrier();
                const int rr = r - rk + lane / L, l = lane % L, t = tl0 + l;
                if (rr <= r && l < nl && t < ttop) {
                    S* dst = level_dst<S>(P, t);
                    const int y = jy0 + rr - t, x = jx0 + bx - 2 - t;
                    const A v0 = myrfs[2 * lane], v1 = myrfs[2 * lane + 1];
                    if (!BND) {
                        Tr<S>::st(dst + (size_t)y * nx + x, v0);
                        Tr<S>::st(dst + (size_t)y * nx + x + 1, v1);
                    } else if (y >= 1 && y <= ny - 2) {
                        if (x >= 1 && x <= nx - 2) Tr<S>::st(dst + (size_t)y * nx + x, v0);
                        if (x + 1 >= 1 && x + 1 <= nx - 2) Tr<S>::st(dst + (size_t)y * nx + x + 1, v1);
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        if constexpr (G > 1) __syncthreads();
    }
}

template <typename S, int C, int L, int G>
__global__ void __launch_bounds__(64 * G) k_tiled2d(TiledLaunch Lc) {
    using A = typename Tr<S>::A;
    __shared__ A hand[(G > 1 ? G - 1 : 1) * 2 * (64 * C + 2)];
    __shared__ A lfs[G * 128];
    __shared__ A rfs[G * 128];
    __shared__ int s_tk;
    __shared__ int s_go;
    // One block per queue entry.  The tile is the block's ticket, not its
    // blockIdx: tickets are handed out in the order blocks start, so every
    // predecessor of a ticket was taken earlier by a block that is running,
    // and the waits below always end.  (A persistent loop around the
    // thread-0 regions below is lowered into per-lane loops that deadlock.)
    const int wave = uni((int)(threadIdx.x >> 6));
    if (threadIdx.x == 0)
        s_tk = (int)__hip_atomic_fetch_add(Lc.hdr + HDR_TICKET, 1u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int tk = uni(s_tk);
    if (tk >= Lc.nq) return;
    const QEntry e = Lc.queue[tk];
    const int pi = Lc.qprob ? uni((int)Lc.qprob[tk]) : 0;
    const TiledProblem P = Lc.probs[pi];
    const int kt = uni((int)e.k[0]), ky = uni((int)e.k[1]), kx = uni((int)e.k[2]);
    unsigned* cnt = P.counters + ((size_t)kt * P.cnt[1] + ky) * P.cnt[2] + kx;
    if (wave == 0) {
        unsigned need = 0;
#pragma unroll
        for (int m = 1; m < 8; ++m)
            need += leaf_nonempty(P, kt - ((m >> 2) & 1), ky - ((m >> 1) & 1), kx - (m & 1));
        const bool go = wait_ready(cnt, need, Lc.hdr, Lc.limit_ticks);
        if (threadIdx.x == 0) s_go = go ? 1 : 0;
    }
    __syncthreads();
    const int go = uni(s_go);
    // every wave acquires: the barrier alone does not order its loads after
    // another wave's cache invalidation
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (go) {
        if (leaf_interior(P, kt, ky, kx))
            exec_tile<S, C, L, G, false>(P, kt, ky, kx, hand, lfs, rfs);
        else
            exec_tile<S, C, L, G, true>(P, kt, ky, kx, hand, lfs, rfs);
    }
    // every wave releases its own stores (the barrier does not wait for
    // outstanding vector-memory stores), then one thread signals
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int m = 1; m < 8; ++m) {
            const int a = (m >> 2) & 1, b = (m >> 1) & 1, c = m & 1;
            if (kt + a < P.cnt[0] && ky + b < P.cnt[1] && kx + c < P.cnt[2])
                signal(cnt + ((size_t)a * P.cnt[1] + b) * P.cnt[2] + c);
        }
    }
}

template <typename S, int C, int L, int G>
hipError_t launch_inst(const TiledLaunch& Lc, int, hipStream_t s) {
    if (Lc.nq <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_tiled2d<S, C, L, G>), dim3(Lc.nq), dim3(64 * G), 0, s, Lc);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_dtype(const int* b, const TiledLaunch& Lc, int grid_cap, hipStream_t s) {
    const int C = b[2] / 64;
    const int bt = b[0];
#define PCOT_TL(CC, LL, GG) \
    if (C == CC && bt <= LL * GG) return launch_inst<S, CC, LL, GG>(Lc, grid_cap, s);
    // levels per wave: 8 for 1-2 columns per lane, 4 for 4 (register budget)
    PCOT_TL(1, 4, 1) PCOT_TL(1, 8, 1) PCOT_TL(1, 8, 2) PCOT_TL(1, 8, 4) PCOT_TL(1, 8, 8)
    PCOT_TL(2, 4, 1) PCOT_TL(2, 8, 1) PCOT_TL(2, 8, 2) PCOT_TL(2, 8, 4) PCOT_TL(2, 8, 8)
    PCOT_TL(4, 4, 1) PCOT_TL(4, 4, 2) PCOT_TL(4, 4, 4) PCOT_TL(4, 4, 8)
#undef PCOT_TL
    return hipErrorInvalidValue;
}

}  // namespace

bool tiled2d_supported(const int* b) {
    // b = {bt, by, bx}
    if (b[2] != 64 && b[2] != 128 && b[2] != 256) return false;
    if (b[1] < 2 || b[1] > 4096) return false;
    if (b[0] < 1 || b[0] > (b[2] == 256 ? 32 : 64)) return false;
    return true;
}

hipError_t launch_tiled2d(int dtype, const int* b, const TiledLaunch& Lc, int grid_cap, hipStream_t s) {
    switch (dtype) {
        case 0: return launch_dtype<double>(b, Lc, grid_cap, s);
        case 1: return launch_dtype<float>(b, Lc, grid_cap, s);
        default: return launch_dtype<uint16_t>(b, Lc, grid_cap, s);
    }
}

}  // namespace pcot
