// Time-skewed tile executor for the 3-point Jacobi-1D stencil.
//
// A leaf is t in [t0, t0+nt) x jx in [jx0, jx0+bx) of the skewed space
// jx = x + t.  Level t at jx updates u_{t+1}[jx-t] from level t-1 outputs at
// l (jx-2), c (jx-1), r (jx) as ((l + c) + r) / 3.
//
// One wave per tile: lane l owns columns jx0 + l*C .. + C-1 (bx = 64*C) and
// the wave steps through the levels; the one- and two-column shifts cross
// lanes with DPP wave_shr:1.  The two-wide left face of every level (written
// by the left neighbour tile) is loaded once at tile start, one level per
// lane, and broadcast with readlane; the two-wide right face of every level is
// gathered the same way into per-level lanes and written with one store.
// Tiles that span more than 64 levels process them in groups of 64.
#include "bufio.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace pcot {

namespace {

__device__ __forceinline__ double rdlane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float rdlane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

template <typename S, int C>
__device__ __forceinline__ void exec1d(const TiledProblem& P, const int* k) {
    using A = typename Tr<S>::A;
    constexpr int ES = sizeof(S);
    const int lane = threadIdx.x & 63;
    const int n = P.n[0], bt = P.b[0];
    const int t0 = k[0] * bt;
    const int nt = min(bt, P.T - t0);
    const int ttop = t0 + nt - 1;
    const int jx0 = 1 + k[1] * (64 * C);
    const int jxl = jx0 + lane * C;
    const uint32_t bytes = (uint32_t)n * ES;
    const uintptr_t pin = (uintptr_t)uptr(P.in), pb0 = (uintptr_t)uptr(P.buf0), pb1 = (uintptr_t)uptr(P.buf1);
    auto src_of = [&](int t) {  // buffer holding u_t
        return make_rsrc(uptr((const void*)pick(pick(pb0, pb1, t), pin, t == 0)), bytes);
    };
    auto dst_of = [&](int t) { return make_rsrc(uptr((const void*)pick(pb0, pb1, t + 1)), bytes); };
    auto ok = [&](int x) { return x >= 1 && x <= n - 2; };
    auto offs = [&](int x) { return x * ES; };  // negative / past-end offsets read 0 (never used)

    // level t0's input row: u_t0[jx - t0 + 1] for jx in [jxl-2, jxl+C)
    A cur[C], xa, xb;
    {
        const rsrc_t r = src_of(t0);
        const int x = jxl - t0 + 1;
        xb = IO<S>::ld(r, offs(x - 2));
        xa = IO<S>::ld(r, offs(x - 1));
#pragma unroll
        for (int c = 0; c < C; ++c) cur[c] = IO<S>::ld(r, offs(x + c));
    }
    for (int g0 = t0; g0 <= ttop; g0 += 64) {
        const int ng = min(64, ttop + 1 - g0);
        // left faces: lane l holds level g0+l's outputs at jx0-2, jx0-1
        A lfB = A(0), lfA = A(0);
        if (lane < ng && g0 + lane < ttop) {
            const int t = g0 + lane;
            const int x = jx0 - 2 - t;
            const rsrc_t rE = dst_of(g0), rO = dst_of(g0 + 1);  // parity of t vs g0
            const bool even = (lane & 1) == 0;
            const A bE = IO<S>::ld(rE, even ? offs(x) : OOB), bO = IO<S>::ld(rO, even ? OOB : offs(x));
            const A aE = IO<S>::ld(rE, even ? offs(x + 1) : OOB), aO = IO<S>::ld(rO, even ? OOB : offs(x + 1));
            lfB = even ? bE : bO;
            lfA = even ? aE : aO;
        }
        A rf0 = A(0), rf1 = A(0);  // right faces gathered per level: lane l <- level g0+l
        for (int i = 0; i < ng; ++i) {
            const int t = g0 + i;
            A out[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const A l_ = c >= 2 ? cur[c - 2] : (c == 1 ? xa : xb);
                const A c_ = c >= 1 ? cur[c - 1] : xa;
                const A r_ = cur[c];
                const A v = Tr<S>::rnd(jac1(l_, c_, r_));
                out[c] = ok(jxl + c - t) ? v : c_;  // boundary cells carried unchanged
            }
            if (t == ttop) {
                const rsrc_t r = dst_of(t);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const int x = jxl + c - t;
                    IO<S>::st(r, ok(x) ? offs(x) : OOB, out[c]);
                }
            } else {
                const A fa = rdlane(lfA, i), fb = rdlane(lfB, i);
                xa = shr1(out[C - 1], fa);
                if constexpr (C >= 2) xb = shr1(out[C >= 2 ? C - 2 : 0], fb);
                else xb = shr1(xa, fb);
                const A h0 = rdlane(C >= 2 ? out[C >= 2 ? C - 2 : 0] : xa, 63), h1 = rdlane(out[C - 1], 63);
                if (lane == i) {
                    rf0 = h0;
                    rf1 = h1;
                }
#pragma unroll
                for (int c = 0; c < C; ++c) cur[c] = out[c];
            }
        }
        // right faces of this group's levels (columns jx0+bx-2, jx0+bx-1)
        if (lane < ng && g0 + lane < ttop) {
            const int t = g0 + lane;
            const int x = jx0 + 64 * C - 2 - t;
            const rsrc_t rE = dst_of(g0), rO = dst_of(g0 + 1);
            const bool even = (lane & 1) == 0;
            IO<S>::st(rE, even && ok(x) ? offs(x) : OOB, rf0);
            IO<S>::st(rO, !even && ok(x) ? offs(x) : OOB, rf0);
            IO<S>::st(rE, even && ok(x + 1) ? offs(x + 1) : OOB, rf1);
            IO<S>::st(rO, !even && ok(x + 1) ? offs(x + 1) : OOB, rf1);
        }
    }
}

template <typename S, int C>
__global__ void __launch_bounds__(64) k_tiled1d(TiledLaunch Lc) {
    __shared__ int s_tk, s_go;
    run_queued_tile<1, true>(Lc, &s_tk, &s_go, [&](const TiledProblem& P, const int* k) { exec1d<S, C>(P, k); });
}

template <typename S>
hipError_t launch_dtype(const int* b, const TiledLaunch& Lc, hipStream_t s) {
    if (Lc.nq <= 0) return hipSuccess;
    switch (b[1]) {
        case 64: hipLaunchKernelGGL((k_tiled1d<S, 1>), dim3(Lc.nq), dim3(64), 0, s, Lc); break;
        case 128: hipLaunchKernelGGL((k_tiled1d<S, 2>), dim3(Lc.nq), dim3(64), 0, s, Lc); break;
        case 256: hipLaunchKernelGGL((k_tiled1d<S, 4>), dim3(Lc.nq), dim3(64), 0, s, Lc); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

bool tiled1d_supported(const int* b) {
    // b = {bt, bx}
    return (b[1] == 64 || b[1] == 128 || b[1] == 256) && b[0] >= 1 && b[0] <= 4096;
}

hipError_t launch_tiled1d(int dtype, const int* b, const TiledLaunch& Lc, int, hipStream_t s) {
    switch (dtype) {
        case 0: return launch_dtype<double>(b, Lc, s);
        case 1: return launch_dtype<float>(b, Lc, s);
        default: return launch_dtype<uint16_t>(b, Lc, s);
    }
}

}  // namespace pcot
