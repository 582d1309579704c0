// Time-skewed tile executor for the 5-point Jacobi-2D stencil.  Blocks take
// tiles from a device queue in schedule order and wait on per-tile dependency
// counters.
//
// A leaf (the base function of the recursive decomposition, Section 4.2, and
// equally one single-level tile, Section 3) is the box
//   t in [t0, t0+nt) x jy in [jy0, jy0+by) x jx in [jx0, jx0+bx)
// of the skewed space jy = y + t, jx = x + t.  Level t at (jy, jx) updates
// u_{t+1}[jy-t][jx-t] from level t-1 outputs at
//   c (jy-1, jx-1), n (jy-2, jx-1), s (jy, jx-1), e (jy-1, jx), w (jy-1, jx-2),
// so inside a tile every input comes from the same or a lower row and column.
//
// Mapping onto CDNA:
//  * lanes own columns: lane l holds jx = jx0 + l*C .. + C-1 (bx = 64*C); the
//    one- and two-column shifts cross lanes with DPP wave_shr:1;
//  * the block streams along jy; compute wave g of G owns levels
//    [g*L, g*L+L) and runs one row behind wave g-1, taking its input row from
//    an LDS handoff (one barrier per row); a tile keeps bt = G*L levels in
//    registers, so each point crosses HBM once per tile, not once per step;
//  * per level, the two previous input rows live in registers;
//  * the bottom plane u_t0 is staged through LDS in chunks of rows loaded by
//    the whole block one chunk ahead; the two-wide left faces of every level
//    (written by the left neighbour tile) are fetched one chunk of rows ahead;
//    the two-wide right faces are staged in LDS and written once per chunk;
//  * all global memory goes through buffer resources: 32-bit offsets, and
//    out-of-range offsets read 0 / drop the store, which clips tiles at the
//    array edge and masks stores without branches.
// Points outside the interior are carried through unchanged (identity), which
// reproduces the fixed boundary; positions outside the array never feed an
// interior point.  Tiles entirely inside the interior take a path with no
// masks at all.
#include "bufio.hpp"
#include "common.hpp"
#include "kernels.hpp"

#include <type_traits>
#include <utility>

namespace pcot {

namespace {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

template <int C, int G> struct Cfg {
    static constexpr int ROW = 64 * C + 2;          // staged row: 2 left-face values + 64*C columns
    static constexpr int KB = G == 1 ? 4 : 8;       // bottom-plane rows per staging chunk
    static constexpr int NPT = (KB * ROW + 64 * G - 1) / (64 * G);
};

// A staged row in LDS: [0], [1] hold columns jx0-2, jx0-1 (the left
// neighbour's faces); tile column q = lane*C + c sits at 2 + c*64 + lane, so
// the 64 lanes touch 64 consecutive words in every access (no bank conflicts).
template <int C> __device__ __forceinline__ int rpos(int q) { return 2 + (q % C) * 64 + q / C; }
// positions of lane's left neighbours jx-2 and jx-1 of its first column
template <int C> __device__ __forceinline__ int rpos_m2(int lane) {
    return C == 1 ? lane : (lane == 0 ? 0 : 1 + (C - 2) * 64 + lane);
}
template <int C> __device__ __forceinline__ int rpos_m1(int lane) {
    return C == 1 ? lane + 1 : (lane == 0 ? 1 : 1 + (C - 1) * 64 + lane);
}

template <typename A, int C, int G> struct Smem {
    // [g]: input rows of wave g (g > 0); parity by step, row of pair (two
    // rows per step only when a lane holds at most two columns)
    A hand[G][2][C <= 2 ? 2 : 1][Cfg<C, G>::ROW];
    A bchunk[2][Cfg<C, G>::KB][Cfg<C, G>::ROW];
    A lfs[G][128];                     // left faces of the current chunk, per wave
    A rfs[G][128];                     // right faces of the current chunk, per wave
    A junk[G][128];                    // sink for the lanes that stage nothing
    int tk, go;
};

template <typename S, int C, int L, int G, bool BND>
__device__ __forceinline__ void exec_tile(const TiledProblem& P, int kt, int ky, int kx,
                                          Smem<typename Tr<S>::A, C, G>& sm) {
    using A = typename Tr<S>::A;
    using CF = Cfg<C, G>;
    constexpr int ES = sizeof(S);
    constexpr int ROW = CF::ROW, KB = CF::KB, NPT = CF::NPT;
    constexpr int K = 64 / L;  // rows per left/right-face chunk
    const int lane = threadIdx.x & 63;
    const int w = uni((int)(threadIdx.x >> 6));
    const int ny = P.n[0], nx = P.n[1], by = P.b[1], bt = P.b[0];
    const int t0 = kt * bt;
    const int nt = min(bt, P.T - t0);
    const int ttop = t0 + nt - 1;
    const int jy0 = 1 + ky * by, jx0 = 1 + kx * (64 * C);
    const int tl0 = t0 + w * L;
    const int nl = clampi(nt - w * L, 0, L);
    const int jxl = jx0 + lane * C;
    const uint32_t bytes = (uint32_t)ny * (uint32_t)nx * ES;
    const uintptr_t pin = (uintptr_t)uptr(P.in), pb0 = (uintptr_t)uptr(P.buf0), pb1 = (uintptr_t)uptr(P.buf1);
    // descriptors are built from a uniform pointer picked first: selecting
    // between two descriptors would be done in VGPRs
    auto src_of = [&](int t) {  // holds u_t
        const uintptr_t b = pick(pb0, pb1, t);
        return make_rsrc(uptr((const void*)pick(b, pin, t == 0)), bytes);
    };
    auto dst_of = [&](int t) {  // receives u_{t+1}
        return make_rsrc(uptr((const void*)pick(pb0, pb1, t + 1)), bytes);
    };
    auto row_ok = [&](int y) { return !BND || (y >= 1 && y <= ny - 2); };
    auto col_ok = [&](int x) { return !BND || (x >= 1 && x <= nx - 2); };
    auto ld = [&](rsrc_t r, int y, int x) -> A {
        // outside the array: offset out of range (reads 0) or another row (never used)
        if (BND && (y < 0 || y >= ny)) return A(0);
        return IO<S>::ld(r, (y * nx + x) * ES);
    };
    auto st = [&](rsrc_t r, int y, int x, bool ok, A v) { IO<S>::st(r, ok ? (y * nx + x) * ES : OOB, v); };

    // per level: the two previous input rows (jy-1, jy-2) and lane-1's last
    // values of them
    A in1[L][C], in2[L][C], x1a[L], x1b[L], x2a[L];
    unsigned colok = 0xFFFFFFFFu;  // BND: bit l*C+c = column c of level l is interior
    if (BND) {
        colok = 0;
#pragma unroll
        for (int l = 0; l < L; ++l)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int x = jxl + c - (tl0 + l);
                colok |= (x >= 1 && x <= nx - 2) ? (1u << (l * C + c)) : 0u;
            }
    }
    A lfp0 = A(0), lfp1 = A(0);  // left-face prefetch: lane -> (row, level)
    // lane i carries (row, level i % L): the level, hence the buffer parity,
    // differs between lanes, so both uniform descriptors are read (one offset
    // out of range) and the right value is selected
    const rsrc_t rdE = dst_of(tl0), rdO = dst_of(tl0 + 1);  // levels tl0 + even / odd l
    const bool lf_even = ((lane % L) & 1) == 0;
    auto lf_fetch = [&](int r0) {
        const int rr = r0 + lane / L, l = lane % L, t = tl0 + l;
        if (rr < by && l < nl && t < ttop) {
            const int y = jy0 + rr - t, x = jx0 - t - 2;
            const int o = (BND && (y < 0 || y >= ny)) ? OOB : (y * nx + x) * ES;
            const A aE = IO<S>::ld(rdE, lf_even ? o : OOB), aO = IO<S>::ld(rdO, lf_even ? OOB : o);
            const A bE = IO<S>::ld(rdE, lf_even ? o + ES : OOB), bO = IO<S>::ld(rdO, lf_even ? OOB : o + ES);
            lfp0 = lf_even ? aE : aO;
            lfp1 = lf_even ? bE : bO;
        }
    };
    A bst[NPT];  // bottom-plane prefetch
    const rsrc_t rbot = src_of(t0);
    auto chunk_fetch = [&](int c) {
        const int bx0 = jx0 - t0 - 1;
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int idx = threadIdx.x + i * 64 * G;
            const int rr = c * KB + idx / ROW;
            if ((KB * ROW) % (64 * G) == 0 || idx < KB * ROW)
                bst[i] = rr < by ? ld(rbot, jy0 + rr - t0 + 1, bx0 + idx % ROW) : A(0);
        }
    };
    auto chunk_store = [&](int c) {
        A* dstc = &sm.bchunk[c & 1][0][0];
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int idx = threadIdx.x + i * 64 * G;
            if ((KB * ROW) % (64 * G) == 0 || idx < KB * ROW) {
                const int p = idx % ROW;
                dstc[idx - p + (p < 2 ? p : rpos<C>(p - 2))] = bst[i];
            }
        }
    };

    auto step = [&](int S_) {
        const int r = S_ - w;
        if (nl > 0 && r >= 0 && r < by) {
            if (r == 0) {
                // history before this wave's first row: input rows jy0-1 and
                // jy0-2; level t's input row jy' holds u_t[jy' - t + 1][jx - t + 1]
#pragma unroll
                for (int l = 0; l < L; ++l) {
                    if (l < nl) {
                        const int t = tl0 + l;
                        const rsrc_t rr_ = src_of(t);
                        const int y1 = jy0 - t, y2 = jy0 - t - 1, x = jxl - t;
                        x1b[l] = ld(rr_, y1, x - 1);
                        x1a[l] = ld(rr_, y1, x);
#pragma unroll
                        for (int c = 0; c < C; ++c) in1[l][c] = ld(rr_, y1, x + 1 + c);
                        x2a[l] = ld(rr_, y2, x);
#pragma unroll
                        for (int c = 0; c < C; ++c) in2[l][c] = ld(rr_, y2, x + 1 + c);
                    }
                }
            }
            const int jy = jy0 + r;
            const int rk = r % K;
            if (rk == 0) {
                sm.lfs[w][2 * lane] = lfp0;
                sm.lfs[w][2 * lane + 1] = lfp1;
                __builtin_amdgcn_wave_barrier();
                lf_fetch(r + K);
            }
            // input row of this wave's first level
            A in0[C], x0a, x0b;
            {
                const A* h = w == 0 ? &sm.bchunk[(r / KB) & 1][r % KB][0] : &sm.hand[w][(S_ - 1) & 1][0][0];
                x0b = h[rpos_m2<C>(lane)];
                x0a = h[rpos_m1<C>(lane)];
#pragma unroll
                for (int c = 0; c < C; ++c) in0[c] = h[2 + c * 64 + lane];
            }
#pragma unroll
            for (int l = 0; l < L; ++l) {
                if (l < nl) {
                    const int t = tl0 + l;
                    const int y = jy - t;
                    A out[C];
                    const bool rok = row_ok(y);
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        const A cc = c >= 1 ? in1[l][c - 1] : x1a[l];
                        const A nn = c >= 1 ? in2[l][c - 1] : x2a[l];
                        const A ss = c >= 1 ? in0[c - 1] : x0a;
                        const A ee = in1[l][c];
                        const A ww = c >= 2 ? in1[l][c - 2] : (c == 1 ? x1a[l] : x1b[l]);
                        A v = Tr<S>::rnd(jac2(cc, nn, ss, ee, ww));
                        if (BND) v = (rok && ((colok >> (l * C + c)) & 1u)) ? v : cc;
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
                    if (t == ttop || r >= by - 2) {
                        // top plane, or one of the two high rows of this level
                        const rsrc_t dr = dst_of(t);
#pragma unroll
                        for (int c = 0; c < C; ++c)
                            st(dr, y, jxl + c - t, rok && ((colok >> (l * C + c)) & 1u), out[c]);
                    }
                    if (t < ttop) {
                        const A lfA = sm.lfs[w][2 * (rk * L + l) + 1];  // column jx0-1
                        const A lfB = sm.lfs[w][2 * (rk * L + l)];      // column jx0-2
                        x0a = shr1(out[C - 1], lfA);
                        if constexpr (C >= 2) x0b = shr1(out[C >= 2 ? C - 2 : 0], lfB);
                        else x0b = shr1(x0a, lfB);
                        if (lane == 63) {
                            sm.rfs[w][2 * (rk * L + l)] = C >= 2 ? out[C >= 2 ? C - 2 : 0] : x0a;
                            sm.rfs[w][2 * (rk * L + l) + 1] = out[C - 1];
                        }
                        if (l + 1 == L && w + 1 < G) {
                            A* h = &sm.hand[w + 1 < G ? w + 1 : 0][S_ & 1][0][0];
#pragma unroll
                            for (int c = 0; c < C; ++c) h[2 + c * 64 + lane] = out[c];
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
                // flush the staged right faces of this chunk: lane i -> (row, level)
                __builtin_amdgcn_wave_barrier();
                const int rr = r - rk + lane / L, l = lane % L, t = tl0 + l;
                if (rr <= r && l < nl && t < ttop) {
                    const int y = jy0 + rr - t, x = jx0 + 64 * C - 2 - t;
                    const bool rok = row_ok(y);
                    const int o0 = (rok && col_ok(x)) ? (y * nx + x) * ES : OOB;
                    const int o1 = (rok && col_ok(x + 1)) ? (y * nx + x + 1) * ES : OOB;
                    const A v0 = sm.rfs[w][2 * lane], v1 = sm.rfs[w][2 * lane + 1];
                    IO<S>::st(rdE, lf_even ? o0 : OOB, v0);
                    IO<S>::st(rdO, lf_even ? OOB : o0, v0);
                    IO<S>::st(rdE, lf_even ? o1 : OOB, v1);
                    IO<S>::st(rdO, lf_even ? OOB : o1, v1);
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        // bottom-plane staging in block-wide step units: chunk c+1 is loaded
        // during chunk c and published to LDS at its last step
        if (S_ % KB == 0 && S_ > 0) chunk_fetch(S_ / KB + 1);
        if (S_ % KB == KB - 1) chunk_store(S_ / KB + 1);
        __syncthreads();
    };

    chunk_fetch(0);
    if (nl > 0) lf_fetch(0);
    chunk_store(0);
    chunk_fetch(1);
    __syncthreads();
    const int nsteps = by + G - 1;
    for (int S_ = 0; S_ < nsteps; ++S_) step(S_);
}

// Lean path for tiles that hold all bt levels (every tile when bt divides
// T).  Same dataflow as exec_tile; per-level conditions are compile-time or
// hoisted to one branch per row step, the two destination buffers are fixed
// per level parity, and the right-face staging is branch-free.
template <typename S, int C, int L, int G, bool BND>
__device__ __forceinline__ void exec_full(const TiledProblem& P, int kt, int ky, int kx,
                                          Smem<typename Tr<S>::A, C, G>& sm) {
    using A = typename Tr<S>::A;
    using CF = Cfg<C, G>;
    constexpr int ES = sizeof(S);
    constexpr int ROW = CF::ROW, KB = CF::KB, NPT = CF::NPT;
    constexpr int K = 64 / L;  // rows per left/right-face chunk
    const int lane = threadIdx.x & 63;
    const int w = uni((int)(threadIdx.x >> 6));
    const int ny = P.n[0], nx = P.n[1], by = P.b[1];
    const int t0 = kt * (G * L);
    const int tl0 = t0 + w * L;
    const int jy0 = 1 + ky * by, jx0 = 1 + kx * (64 * C);
    const int jxl = jx0 + lane * C;
    const bool topwave = w == G - 1;  // owns the tile's top level
    const uint32_t bytes = (uint32_t)ny * (uint32_t)nx * ES;
    const uintptr_t pin = (uintptr_t)uptr(P.in), pb0 = (uintptr_t)uptr(P.buf0), pb1 = (uintptr_t)uptr(P.buf1);
    // level tl0+l writes u_{tl0+l+1}: buffer parity (tl0 + l + 1) & 1
    const rsrc_t rdE = make_rsrc(uptr((const void*)pick(pb0, pb1, tl0 + 1)), bytes);  // even l
    const rsrc_t rdO = make_rsrc(uptr((const void*)pick(pb0, pb1, tl0)), bytes);      // odd l
    const rsrc_t rbot = make_rsrc(uptr((const void*)pick(pick(pb0, pb1, t0), pin, t0 == 0)), bytes);
    auto offs = [&](int y, int x) { return (y * nx + x) * ES; };
    auto okoff = [&](int y, int x) {  // byte offset, or OOB outside the interior
        return (!BND || (y >= 1 && y <= ny - 2 && x >= 1 && x <= nx - 2)) ? offs(y, x) : OOB;
    };
    auto ldv = [&](rsrc_t r, int y, int x) -> A {
        if (BND && (y < 0 || y >= ny)) return A(0);
        return IO<S>::ld(r, offs(y, x));
    };

    // Input rows of every level in three register banks used in rotation:
    // at step S_ bank S_ % 3 receives the new row, bank (S_ + 2) % 3 holds the
    // row before it and bank (S_ + 1) % 3 the one before that, so rows move on
    // without register copies (the step loop is unrolled by three).  Per bank:
    // the lane's C columns, and the values at jx-1 and jx-2 (lane-1's last
    // two columns, or the left faces for lane 0).
    A H[L][3][C], XA[L][3], XB[L][3];
    // history before the first row (step w): input rows jy0-1 and jy0-2 of
    // every level; level t's input row jy' holds u_t[jy' - t + 1][jx - t + 1]
    auto load_hist = [&](auto b1c, auto b2c) {
        constexpr int B1 = decltype(b1c)::value, B2 = decltype(b2c)::value;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const int t = tl0 + l;
            const uintptr_t ps = pick(pick(pb0, pb1, t), pin, t == 0);
            const rsrc_t rs = make_rsrc(uptr((const void*)ps), bytes);
            const int y1 = jy0 - t, y2 = jy0 - t - 1, x = jxl - t;
            XB[l][B1] = ldv(rs, y1, x - 1);
            XA[l][B1] = ldv(rs, y1, x);
#pragma unroll
            for (int c = 0; c < C; ++c) H[l][B1][c] = ldv(rs, y1, x + 1 + c);
            XA[l][B2] = ldv(rs, y2, x);
            XB[l][B2] = A(0);  // never read: jx-2 is used only from the previous row
#pragma unroll
            for (int c = 0; c < C; ++c) H[l][B2][c] = ldv(rs, y2, x + 1 + c);
        }
    };
    switch (w % 3) {  // the first row of wave w is computed at step w
        case 0: load_hist(std::integral_constant<int, 2>{}, std::integral_constant<int, 1>{}); break;
        case 1: load_hist(std::integral_constant<int, 0>{}, std::integral_constant<int, 2>{}); break;
        default: load_hist(std::integral_constant<int, 1>{}, std::integral_constant<int, 0>{}); break;
    }
    unsigned colok = 0xFFFFFFFFu;  // BND: bit l*C+c = column c of level l is interior
    if (BND) {
        colok = 0;
#pragma unroll
        for (int l = 0; l < L; ++l)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int x = jxl + c - (tl0 + l);
                colok |= (x >= 1 && x <= nx - 2) ? (1u << (l * C + c)) : 0u;
            }
    }

    // left faces of level tl0+l (its outputs at jx0-2, jx0-1), one chunk of
    // rows ahead; lane i carries (row r0 + i / L, level i % L).  Both buffers
    // are read (one offset out of range) so the descriptor stays uniform.
    // The two candidate loads stay in registers until the chunk is
    // published: selecting right after the loads would wait for them.
    A lfE0 = A(0), lfO0 = A(0), lfE1 = A(0), lfO1 = A(0);
    const int lf_l = lane % L;
    const bool lf_even = (lf_l & 1) == 0;
    const bool lf_top = topwave && lf_l == L - 1;  // the tile's top level has no consumer
    auto lf_fetch = [&](int r0) {
        const int rr = r0 + lane / L, t = tl0 + lf_l;
        const int y = jy0 + rr - t, x = jx0 - t - 2;
        const bool ok = rr < by && !lf_top && (!BND || (y >= 0 && y < ny));
        const int o = ok ? offs(y, x) : OOB;
        lfE0 = IO<S>::ld(rdE, lf_even ? o : OOB);
        lfO0 = IO<S>::ld(rdO, lf_even ? OOB : o);
        lfE1 = IO<S>::ld(rdE, lf_even ? o + ES : OOB);
        lfO1 = IO<S>::ld(rdO, lf_even ? OOB : o + ES);
    };
    A bst[NPT];
    auto chunk_fetch = [&](int c) {
        const int bx0 = jx0 - t0 - 1;
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int idx = threadIdx.x + i * 64 * G;
            const int rr = c * KB + idx / ROW;
            if ((KB * ROW) % (64 * G) == 0 || idx < KB * ROW)
                bst[i] = rr < by ? ldv(rbot, jy0 + rr - t0 + 1, bx0 + idx % ROW) : A(0);
        }
    };
    auto chunk_store = [&](int c) {
        A* dstc = &sm.bchunk[c & 1][0][0];
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int idx = threadIdx.x + i * 64 * G;
            if ((KB * ROW) % (64 * G) == 0 || idx < KB * ROW) {
                const int p = idx % ROW;
                dstc[idx - p + (p < 2 ? p : rpos<C>(p - 2))] = bst[i];
            }
        }
    };
    // right-face staging target: lane 63 writes the chunk slot, others a sink
    A* const rf_base = lane == 63 ? &sm.rfs[w][0] : &sm.junk[w][2 * lane];
    const int rf_stride = lane == 63 ? 2 : 0;

    // all levels of one row step at step phase PH = S_ % 3; TAIL: one of the
    // tile's two last rows, where every level also writes its row (the
    // two-wide high face)
    auto levels = [&](auto tail, auto ph, int S_, int r, int rk) {
        constexpr bool TAIL = decltype(tail)::value;
        constexpr int P0 = decltype(ph)::value, P1 = (P0 + 2) % 3, P2 = (P0 + 1) % 3;  // new, previous, before
        const int jy = jy0 + r;
        {
            const A* h = w == 0 ? &sm.bchunk[(r / KB) & 1][r % KB][0] : &sm.hand[w][(S_ - 1) & 1][0][0];
            XB[0][P0] = h[rpos_m2<C>(lane)];
            XA[0][P0] = h[rpos_m1<C>(lane)];
#pragma unroll
            for (int c = 0; c < C; ++c) H[0][P0][c] = h[2 + c * 64 + lane];
        }
        // left faces of every level for this row, read before any LDS write of
        // the step so that they are off the level-to-level dependency chain
        A lfa[L], lfb[L];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            lfa[l] = sm.lfs[w][2 * (rk * L + l) + 1];  // column jx0-1
            lfb[l] = sm.lfs[w][2 * (rk * L + l)];      // column jx0-2
        }
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const int t = tl0 + l;
            const int y = jy - t;
            const bool rok = !BND || (y >= 1 && y <= ny - 2);
            A out[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const A cc = c >= 1 ? H[l][P1][c - 1] : XA[l][P1];
                const A nn = c >= 1 ? H[l][P2][c - 1] : XA[l][P2];
                const A ss = c >= 1 ? H[l][P0][c - 1] : XA[l][P0];
                const A ee = H[l][P1][c];
                const A ww = c >= 2 ? H[l][P1][c - 2] : (c == 1 ? XA[l][P1] : XB[l][P1]);
                A v = Tr<S>::rnd(jac2(cc, nn, ss, ee, ww));
                if (BND) v = (rok && ((colok >> (l * C + c)) & 1u)) ? v : cc;
                out[c] = v;
            }
            const rsrc_t rd = (l & 1) ? rdO : rdE;
            auto store_row = [&]() {
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const int x = jxl + c - t;
                    IO<S>::st(rd, BND ? ((rok && ((colok >> (l * C + c)) & 1u)) ? offs(y, x) : OOB) : offs(y, x), out[c]);
                }
            };
            // out is the next level's new input row: its values at jx-1 and
            // jx-2 come from lane-1 (left faces for lane 0)
            auto pass_on = [&](A& xa, A& xb) {
                xa = shr1(out[C - 1], lfa[l]);
                if constexpr (C >= 2) xb = shr1(out[C >= 2 ? C - 2 : 0], lfb[l]);
                else xb = shr1(xa, lfb[l]);
                A* rf = rf_base + rf_stride * (rk * L + l);
                rf[0] = C >= 2 ? out[C >= 2 ? C - 2 : 0] : xa;
                rf[1] = out[C - 1];
                if (TAIL) store_row();
            };
            if (l + 1 < L) {
                pass_on(XA[l + 1 < L ? l + 1 : 0][P0], XB[l + 1 < L ? l + 1 : 0][P0]);
#pragma unroll
                for (int c = 0; c < C; ++c) H[l + 1 < L ? l + 1 : 0][P0][c] = out[c];
            } else if (!topwave) {
                A xa, xb;
                pass_on(xa, xb);
                A* h = &sm.hand[w + 1 < G ? w + 1 : 0][S_ & 1][0][0];
#pragma unroll
                for (int c = 0; c < C; ++c) h[2 + c * 64 + lane] = out[c];
                if (lane == 0) {
                    h[0] = lfb[l];
                    h[1] = lfa[l];
                }
            } else {
                store_row();  // top plane
            }
        }
    };

    chunk_fetch(0);
    lf_fetch(0);
    chunk_store(0);
    chunk_fetch(1);
    __syncthreads();
    const int nsteps = by + G - 1;
    auto step = [&](auto ph, int S_) {
        if (S_ % KB == 0 && S_ > 0) {
            // publish chunk c = S_/KB (loaded during chunk c-1) before any
            // store of this step, then start loading chunk c+1
            chunk_store(S_ / KB);
            __syncthreads();
            chunk_fetch(S_ / KB + 1);
        }
        const int r = S_ - w;
        if (r >= 0 && r < by) {
            const int rk = r % K;
            if (rk == 0) {
                sm.lfs[w][2 * lane] = lf_even ? lfE0 : lfO0;
                sm.lfs[w][2 * lane + 1] = lf_even ? lfE1 : lfO1;
                __builtin_amdgcn_wave_barrier();
                lf_fetch(r + K);
            }
            if (r < by - 2) levels(std::integral_constant<bool, false>{}, ph, S_, r, rk);
            else levels(std::integral_constant<bool, true>{}, ph, S_, r, rk);
            if (rk == K - 1 || r == by - 1) {
                // flush the staged right faces of this chunk: lane i -> (row, level)
                __builtin_amdgcn_wave_barrier();
                const int rr = r - rk + lane / L, t = tl0 + lf_l;
                const int y = jy0 + rr - t, x = jx0 + 64 * C - 2 - t;
                const bool ok = rr <= r && !lf_top;
                const rsrc_t r0 = rdE, r1 = rdO;
                const int o0 = ok ? okoff(y, x) : OOB, o1 = ok ? okoff(y, x + 1) : OOB;
                const A v0 = sm.rfs[w][2 * lane], v1 = sm.rfs[w][2 * lane + 1];
                IO<S>::st(r0, lf_even ? o0 : OOB, v0);
                IO<S>::st(r1, lf_even ? OOB : o0, v0);
                IO<S>::st(r0, lf_even ? o1 : OOB, v1);
                IO<S>::st(r1, lf_even ? OOB : o1, v1);
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();
    };
    for (int S0 = 0; S0 < nsteps; S0 += 3) {
        step(std::integral_constant<int, 0>{}, S0);
        if (S0 + 1 < nsteps) step(std::integral_constant<int, 1>{}, S0 + 1);
        if (S0 + 2 < nsteps) step(std::integral_constant<int, 2>{}, S0 + 2);
    }
}

// Full tiles with an even number of rows: like exec_full, but every step
// advances two rows (a pair), which halves the steps, barriers and LDS
// hand-offs per update.  Row B of a pair reads row A of the same level as its
// north/centre neighbours, so within a level the pair is computed A then B
// from registers.
template <typename S, int C, int L, int G, bool BND>
__device__ __forceinline__ void exec_pair(const TiledProblem& P, int kt, int ky, int kx,
                                          Smem<typename Tr<S>::A, C, G>& sm) {
    using A = typename Tr<S>::A;
    using CF = Cfg<C, G>;
    constexpr int ES = sizeof(S);
    constexpr int ROW = CF::ROW, KB = CF::KB, NPT = CF::NPT;
    constexpr int K = 64 / L;  // rows per left/right-face chunk (even)
    static_assert(K % 2 == 0 && KB % 2 == 0, "chunks hold whole pairs");
    const int lane = threadIdx.x & 63;
    const int w = uni((int)(threadIdx.x >> 6));
    const int ny = P.n[0], nx = P.n[1], by = P.b[1];
    const int t0 = kt * (G * L);
    const int tl0 = t0 + w * L;
    const int jy0 = 1 + ky * by, jx0 = 1 + kx * (64 * C);
    const int jxl = jx0 + lane * C;
    const bool topwave = w == G - 1;
    const uint32_t bytes = (uint32_t)ny * (uint32_t)nx * ES;
    const uintptr_t pin = (uintptr_t)uptr(P.in), pb0 = (uintptr_t)uptr(P.buf0), pb1 = (uintptr_t)uptr(P.buf1);
    const rsrc_t rdE = make_rsrc(uptr((const void*)pick(pb0, pb1, tl0 + 1)), bytes);  // even l
    const rsrc_t rdO = make_rsrc(uptr((const void*)pick(pb0, pb1, tl0)), bytes);      // odd l
    const rsrc_t rbot = make_rsrc(uptr((const void*)pick(pick(pb0, pb1, t0), pin, t0 == 0)), bytes);
    auto offs = [&](int y, int x) { return (y * nx + x) * ES; };
    auto okoff = [&](int y, int x) {
        return (!BND || (y >= 1 && y <= ny - 2 && x >= 1 && x <= nx - 2)) ? offs(y, x) : OOB;
    };
    auto ldv = [&](rsrc_t r, int y, int x) -> A {
        if (BND && (y < 0 || y >= ny)) return A(0);
        return IO<S>::ld(r, offs(y, x));
    };

    A in1[L][C], in2[L][C], x1a[L], x1b[L], x2a[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const int t = tl0 + l;
        const uintptr_t ps = pick(pick(pb0, pb1, t), pin, t == 0);
        const rsrc_t rs = make_rsrc(uptr((const void*)ps), bytes);
        const int y1 = jy0 - t, y2 = jy0 - t - 1, x = jxl - t;
        x1b[l] = ldv(rs, y1, x - 1);
        x1a[l] = ldv(rs, y1, x);
#pragma unroll
        for (int c = 0; c < C; ++c) in1[l][c] = ldv(rs, y1, x + 1 + c);
        x2a[l] = ldv(rs, y2, x);
#pragma unroll
        for (int c = 0; c < C; ++c) in2[l][c] = ldv(rs, y2, x + 1 + c);
    }
    unsigned colok = 0xFFFFFFFFu;
    if (BND) {
        colok = 0;
#pragma unroll
        for (int l = 0; l < L; ++l)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int x = jxl + c - (tl0 + l);
                colok |= (x >= 1 && x <= nx - 2) ? (1u << (l * C + c)) : 0u;
            }
    }

    A lfE0 = A(0), lfO0 = A(0), lfE1 = A(0), lfO1 = A(0);
    const int lf_l = lane % L;
    const bool lf_even = (lf_l & 1) == 0;
    const bool lf_top = topwave && lf_l == L - 1;
    auto lf_fetch = [&](int r0) {
        const int rr = r0 + lane / L, t = tl0 + lf_l;
        const int y = jy0 + rr - t, x = jx0 - t - 2;
        const bool ok = rr < by && !lf_top && (!BND || (y >= 0 && y < ny));
        const int o = ok ? offs(y, x) : OOB;
        lfE0 = IO<S>::ld(rdE, lf_even ? o : OOB);
        lfO0 = IO<S>::ld(rdO, lf_even ? OOB : o);
        lfE1 = IO<S>::ld(rdE, lf_even ? o + ES : OOB);
        lfO1 = IO<S>::ld(rdO, lf_even ? OOB : o + ES);
    };
    A bst[NPT];
    auto chunk_fetch = [&](int c) {
        const int bx0 = jx0 - t0 - 1;
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int idx = threadIdx.x + i * 64 * G;
            const int rr = c * KB + idx / ROW;
            if ((KB * ROW) % (64 * G) == 0 || idx < KB * ROW)
                bst[i] = rr < by ? ldv(rbot, jy0 + rr - t0 + 1, bx0 + idx % ROW) : A(0);
        }
    };
    auto chunk_store = [&](int c) {
        A* dstc = &sm.bchunk[c & 1][0][0];
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int idx = threadIdx.x + i * 64 * G;
            if ((KB * ROW) % (64 * G) == 0 || idx < KB * ROW) {
                const int p = idx % ROW;
                dstc[idx - p + (p < 2 ? p : rpos<C>(p - 2))] = bst[i];
            }
        }
    };
    A* const rf_base = lane == 63 ? &sm.rfs[w][0] : &sm.junk[w][2 * lane];
    const int rf_stride = lane == 63 ? 2 : 0;

    // all levels of one pair of rows (rA = 2*p, rA+1); TAIL: the tile's last
    // pair, where every level also writes both rows (two-wide high face)
    auto levels = [&](auto tail, int S_, int rA, int rk) {
        constexpr bool TAIL = decltype(tail)::value;
        A a0[C], b0[C], a0a, a0b, b0a, b0b;  // level input rows A, B and lane-1's last values
        {
            const A* hA = w == 0 ? &sm.bchunk[(rA / KB) & 1][rA % KB][0] : &sm.hand[w][(S_ - 1) & 1][0][0];
            const A* hB = w == 0 ? &sm.bchunk[(rA / KB) & 1][rA % KB + 1][0] : &sm.hand[w][(S_ - 1) & 1][1][0];
            a0b = hA[rpos_m2<C>(lane)];
            a0a = hA[rpos_m1<C>(lane)];
            b0b = hB[rpos_m2<C>(lane)];
            b0a = hB[rpos_m1<C>(lane)];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                a0[c] = hA[2 + c * 64 + lane];
                b0[c] = hB[2 + c * 64 + lane];
            }
        }
        A lfaA[L], lfbA[L], lfaB[L], lfbB[L];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            lfaA[l] = sm.lfs[w][2 * (rk * L + l) + 1];
            lfbA[l] = sm.lfs[w][2 * (rk * L + l)];
            lfaB[l] = sm.lfs[w][2 * ((rk + 1) * L + l) + 1];
            lfbB[l] = sm.lfs[w][2 * ((rk + 1) * L + l)];
        }
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const int t = tl0 + l;
            const int yA = jy0 + rA - t, yB = yA + 1;
            const bool okA = !BND || (yA >= 1 && yA <= ny - 2);
            const bool okB = !BND || (yB >= 1 && yB <= ny - 2);
            A oa[C], ob[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                // row A: c (rA-1, jx-1), n (rA-2, jx-1), s (rA, jx-1), e (rA-1, jx), w (rA-1, jx-2)
                const A cc = c >= 1 ? in1[l][c - 1] : x1a[l];
                const A nn = c >= 1 ? in2[l][c - 1] : x2a[l];
                const A ss = c >= 1 ? a0[c - 1] : a0a;
                const A ww = c >= 2 ? in1[l][c - 2] : (c == 1 ? x1a[l] : x1b[l]);
                A v = Tr<S>::rnd(jac2(cc, nn, ss, in1[l][c], ww));
                if (BND) v = (okA && ((colok >> (l * C + c)) & 1u)) ? v : cc;
                oa[c] = v;
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                // row B: c (rA, jx-1), n (rA-1, jx-1), s (rB, jx-1), e (rA, jx), w (rA, jx-2)
                const A cc = c >= 1 ? a0[c - 1] : a0a;
                const A nn = c >= 1 ? in1[l][c - 1] : x1a[l];
                const A ss = c >= 1 ? b0[c - 1] : b0a;
                const A ww = c >= 2 ? a0[c - 2] : (c == 1 ? a0a : a0b);
                A v = Tr<S>::rnd(jac2(cc, nn, ss, a0[c], ww));
                if (BND) v = (okB && ((colok >> (l * C + c)) & 1u)) ? v : cc;
                ob[c] = v;
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                in2[l][c] = a0[c];
                in1[l][c] = b0[c];
            }
            x2a[l] = a0a;
            x1a[l] = b0a;
            x1b[l] = b0b;
            const rsrc_t rd = (l & 1) ? rdO : rdE;
            auto store_rows = [&]() {
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const int x = jxl + c - t;
                    const bool cok = (colok >> (l * C + c)) & 1u;
                    IO<S>::st(rd, BND ? ((okA && cok) ? offs(yA, x) : OOB) : offs(yA, x), oa[c]);
                    IO<S>::st(rd, BND ? ((okB && cok) ? offs(yB, x) : OOB) : offs(yB, x), ob[c]);
                }
            };
            if (l + 1 < L || !topwave) {
                const A na = shr1(oa[C - 1], lfaA[l]), nb = shr1(ob[C - 1], lfaB[l]);
                A nab, nbb;
                if constexpr (C >= 2) {
                    nab = shr1(oa[C >= 2 ? C - 2 : 0], lfbA[l]);
                    nbb = shr1(ob[C >= 2 ? C - 2 : 0], lfbB[l]);
                } else {
                    nab = shr1(na, lfbA[l]);
                    nbb = shr1(nb, lfbB[l]);
                }
                A* rf = rf_base + rf_stride * (rk * L + l);
                rf[0] = C >= 2 ? oa[C >= 2 ? C - 2 : 0] : na;
                rf[1] = oa[C - 1];
                A* rfb = rf_base + rf_stride * ((rk + 1) * L + l);
                rfb[0] = C >= 2 ? ob[C >= 2 ? C - 2 : 0] : nb;
                rfb[1] = ob[C - 1];
                if (TAIL) store_rows();
                if (l + 1 < L) {
                    a0a = na;
                    a0b = nab;
                    b0a = nb;
                    b0b = nbb;
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        a0[c] = oa[c];
                        b0[c] = ob[c];
                    }
                } else {
                    A* hA = &sm.hand[w + 1 < G ? w + 1 : 0][S_ & 1][0][0];
                    A* hB = &sm.hand[w + 1 < G ? w + 1 : 0][S_ & 1][1][0];
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        hA[2 + c * 64 + lane] = oa[c];
                        hB[2 + c * 64 + lane] = ob[c];
                    }
                    if (lane == 0) {
                        hA[0] = lfbA[l];
                        hA[1] = lfaA[l];
                        hB[0] = lfbB[l];
                        hB[1] = lfaB[l];
                    }
                }
            } else {
                store_rows();  // top plane
            }
        }
    };

    chunk_fetch(0);
    lf_fetch(0);
    chunk_store(0);
    chunk_fetch(1);
    __syncthreads();
    const int npairs = by / 2;
    const int nsteps = npairs + G - 1;
    constexpr int KP = KB / 2;  // pairs per bottom-plane chunk
    for (int S_ = 0; S_ < nsteps; ++S_) {
        if (S_ % KP == 0 && S_ > 0) {
            chunk_store(S_ / KP);
            __syncthreads();
            chunk_fetch(S_ / KP + 1);
        }
        const int pr = S_ - w;
        if (pr >= 0 && pr < npairs) {
            const int rA = 2 * pr;
            const int rk = rA % K;
            if (rk == 0) {
                sm.lfs[w][2 * lane] = lf_even ? lfE0 : lfO0;
                sm.lfs[w][2 * lane + 1] = lf_even ? lfE1 : lfO1;
                __builtin_amdgcn_wave_barrier();
                lf_fetch(rA + K);
            }
            if (pr < npairs - 1) levels(std::integral_constant<bool, false>{}, S_, rA, rk);
            else levels(std::integral_constant<bool, true>{}, S_, rA, rk);
            if (rk + 1 == K - 1 || rA + 1 == by - 1) {
                __builtin_amdgcn_wave_barrier();
                const int rB = rA + 1;
                const int rr = rB - (rk + 1) + lane / L, t = tl0 + lf_l;
                const int y = jy0 + rr - t, x = jx0 + 64 * C - 2 - t;
                const bool ok = rr <= rB && !lf_top;
                const int o0 = ok ? okoff(y, x) : OOB, o1 = ok ? okoff(y, x + 1) : OOB;
                const A v0 = sm.rfs[w][2 * lane], v1 = sm.rfs[w][2 * lane + 1];
                IO<S>::st(rdE, lf_even ? o0 : OOB, v0);
                IO<S>::st(rdO, lf_even ? OOB : o0, v0);
                IO<S>::st(rdE, lf_even ? o1 : OOB, v1);
                IO<S>::st(rdO, lf_even ? OOB : o1, v1);
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();
    }
}

template <typename S, int C, int L, int G>
__global__ void __launch_bounds__(64 * G) k_tiled2d(TiledLaunch Lc) {
    // two rows per step pays off when a lane holds few columns (measured:
    // faster for b_x = 64, 128; slower for 256, whose registers then spill)
    constexpr bool PAIR = C <= 2;
    using A = typename Tr<S>::A;
    __shared__ Smem<A, C, G> sm;
    run_queued_tile<2, true>(Lc, &sm.tk, &sm.go, [&](const TiledProblem& P, const int* k) {
        const int kt = k[0], ky = k[1], kx = k[2];
        const bool full = (kt + 1) * P.b[0] <= P.T && P.b[0] == G * L;
        if (full && PAIR && (P.b[1] & 1) == 0) {
            if (tile_interior<2>(P, k))
                exec_pair<S, C, L, G, false>(P, kt, ky, kx, sm);
            else
                exec_pair<S, C, L, G, true>(P, kt, ky, kx, sm);
        } else if (full) {
            if (tile_interior<2>(P, k))
                exec_full<S, C, L, G, false>(P, kt, ky, kx, sm);
            else
                exec_full<S, C, L, G, true>(P, kt, ky, kx, sm);
        } else {
            exec_tile<S, C, L, G, true>(P, kt, ky, kx, sm);
        }
    });
}

template <typename S, int C, int L, int G>
hipError_t launch_inst(const TiledLaunch& Lc, hipStream_t s) {
    if (Lc.nq <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_tiled2d<S, C, L, G>), dim3(Lc.nq), dim3(64 * G), 0, s, Lc);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_dtype(const int* b, const TiledLaunch& Lc, hipStream_t s) {
    const int C = b[2] / 64;
    const int bt = b[0];
#define PCOT_TL(CC, LL, GG) \
    if (C == CC && bt <= LL * GG) return launch_inst<S, CC, LL, GG>(Lc, s);
    // levels per wave: 8 for 1-2 columns per lane, 4 for 4 (register budget);
    // for 4 columns and b_t in (8, 16], 8 waves of 2 levels (measured faster
    // than 4 waves of 4: a shorter level chain per step)
    PCOT_TL(1, 4, 1) PCOT_TL(1, 8, 1) PCOT_TL(1, 8, 2) PCOT_TL(1, 8, 4) PCOT_TL(1, 8, 8)
    PCOT_TL(2, 4, 1) PCOT_TL(2, 8, 1) PCOT_TL(2, 8, 2) PCOT_TL(2, 8, 4) PCOT_TL(2, 8, 8)
    PCOT_TL(4, 4, 1) PCOT_TL(4, 4, 2) PCOT_TL(4, 2, 8) PCOT_TL(4, 4, 8)
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

hipError_t launch_tiled2d(int dtype, const int* b, const TiledLaunch& Lc, int, hipStream_t s) {
    switch (dtype) {
        case 0: return launch_dtype<double>(b, Lc, s);
        case 1: return launch_dtype<float>(b, Lc, s);
        default: return launch_dtype<uint16_t>(b, Lc, s);
    }
}

}  // namespace pcot
