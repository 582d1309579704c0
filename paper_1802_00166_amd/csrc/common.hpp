// Shared device helpers: storage types, exact bf16 conversion, wave shifts,
// the persistent-queue protocol and the device header layout.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "kernels.hpp"

namespace pcot {

// ------------------------------------------------------------ storage ---
// S = storage type, A = arithmetic type.  bf16 is stored as its 16-bit
// pattern; loads widen exactly, stores round to nearest even.
template <typename S> struct Tr;
template <> struct Tr<double> {
    using A = double;
    static __device__ __forceinline__ A ld(const double* p) { return *p; }
    static __device__ __forceinline__ void st(double* p, A v) { *p = v; }
    static __device__ __forceinline__ A rnd(A v) { return v; }
};
template <> struct Tr<float> {
    using A = float;
    static __device__ __forceinline__ A ld(const float* p) { return *p; }
    static __device__ __forceinline__ void st(float* p, A v) { *p = v; }
    static __device__ __forceinline__ A rnd(A v) { return v; }
};
__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __uint_as_float(((uint32_t)h) << 16);
}
// Round to nearest, ties to even; a NaN keeps its sign and upper payload
// and is made quiet ((bits >> 16) | 0x40).  gfx950's conversion instruction
// (v_cvt_pk_bf16_f32, emitted for the __bf16 conversion) implements exactly
// this rule, in one instruction instead of six.
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}
template <> struct Tr<uint16_t> {
    using A = float;
    static __device__ __forceinline__ A ld(const uint16_t* p) { return bf16_to_f32(*p); }
    static __device__ __forceinline__ void st(uint16_t* p, A v) { *p = f32_to_bf16(v); }
    static __device__ __forceinline__ A rnd(A v) { return bf16_to_f32(f32_to_bf16(v)); }
};

// ------------------------------------------------------ update rules ---
// Operation order is part of the contract (no FMA: built with
// -ffp-contract=off).
__device__ __forceinline__ double jac1(double l, double c, double r) { return ((l + c) + r) / 3.0; }
__device__ __forceinline__ float jac1(float l, float c, float r) { return ((l + c) + r) / 3.0f; }
__device__ __forceinline__ double jac2(double c, double n, double s, double e, double w) {
    return 0.2 * ((((c + n) + s) + e) + w);
}
__device__ __forceinline__ float jac2(float c, float n, float s, float e, float w) {
    return 0.2f * ((((c + n) + s) + e) + w);
}
__device__ __forceinline__ double heat3(double u, double xp, double xm, double yp, double ym,
                                        double zp, double zm) {
    const double dx = (xp - 2.0 * u) + xm;
    const double dy = (yp - 2.0 * u) + ym;
    const double dz = (zp - 2.0 * u) + zm;
    return u + 0.125 * ((dx + dy) + dz);
}
__device__ __forceinline__ float heat3(float u, float xp, float xm, float yp, float ym, float zp,
                                       float zm) {
    const float dx = (xp - 2.0f * u) + xm;
    const float dy = (yp - 2.0f * u) + ym;
    const float dz = (zp - 2.0f * u) + zm;
    return u + 0.125f * ((dx + dy) + dz);
}

// ------------------------------------------------------- wave shifts ---
// Value of lane-1 (DPP wave_shr:1); lane 0 receives `fill`.
__device__ __forceinline__ float shr1(float v, float fill) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(fill), __float_as_int(v),
                                                      0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ double shr1(double v, double fill) {
    const long long vi = __double_as_longlong(v), fi = __double_as_longlong(fill);
    const int lo = __builtin_amdgcn_update_dpp((int)fi, (int)vi, 0x138, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(fi >> 32), (int)(vi >> 32), 0x138, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// -------------------------------------------- persistent queue protocol ---
__device__ __forceinline__ unsigned ld_relaxed(const unsigned* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-uniform value (an SGPR): branches on it are scalar, so the compiler
// cannot turn block-level control flow into divergent per-lane loops.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ unsigned uni(unsigned v) { return (unsigned)__builtin_amdgcn_readfirstlane((int)v); }

// Spin until *cnt >= need.  Executed by all 64 lanes of one wave with a
// wave-uniform loop condition.  Bounded by a wall-clock limit; on expiry sets
// the error word and the abort flag so that every block drains.  Returns
// false when the tile must be skipped.
__device__ __forceinline__ bool wait_ready(const unsigned* cnt, unsigned need, unsigned* hdr,
                                           long long limit_ticks) {
    if (need > 0 && uni(ld_relaxed(cnt)) < need) {
        const long long t0 = wall_clock64();
        while (uni(ld_relaxed(cnt)) < need) {
            if (uni(ld_relaxed(hdr + HDR_ABORT))) return false;
            if (wall_clock64() - t0 > limit_ticks) {
                if ((threadIdx.x & 63) == 0) {
                    __hip_atomic_store(hdr + HDR_ERROR, DEVERR_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(hdr + HDR_ABORT, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                return false;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    return uni(ld_relaxed(hdr + HDR_ABORT)) == 0u;
}

__device__ __forceinline__ void signal(unsigned* cnt) {
    __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Does tile k (k[0] time, k[1..D] spatial, outer to inner) of problem P hold
// a point of the skewed domain 0 <= t < T, 1 + t <= j_d <= n_d - 2 + t ?
template <int D>
__device__ __forceinline__ bool tile_nonempty(const TiledProblem& P, const int* k) {
#pragma unroll
    for (int i = 0; i <= D; ++i)
        if (k[i] < 0 || k[i] >= P.cnt[i]) return false;
    const int tlo = k[0] * P.b[0];
    int tmin = tlo, tmax = min(tlo + P.b[0] - 1, P.T - 1);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const int lo = 1 + k[i + 1] * P.b[i + 1];
        tmin = max(tmin, lo - P.n[i] + 2);
        tmax = min(tmax, lo + P.b[i + 1] - 2);
    }
    return tmin <= tmax;
}

// Does every level of tile k keep all its points inside the interior?
template <int D>
__device__ __forceinline__ bool tile_interior(const TiledProblem& P, const int* k) {
    const int t0 = k[0] * P.b[0];
    const int t1 = t0 + min(P.b[0], P.T - t0) - 1;
    bool in = true;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const int lo = 1 + k[i + 1] * P.b[i + 1];
        in = in && (lo - t1 >= 1) && (lo + P.b[i + 1] - 1 - t0 <= P.n[i] - 2);
    }
    return in;
}

__device__ __forceinline__ size_t tile_index(const TiledProblem& P, const int* k, int D) {
    size_t idx = 0;
    for (int i = 0; i <= D; ++i) idx = idx * P.cnt[i] + k[i];
    return idx;
}

// One tile of the device queue, run by the calling block:
//  1. take a ticket (the tile is the ticket, not blockIdx: tickets are taken
//     in the order blocks start, so every predecessor of a ticket belongs to
//     a block that is already running and the waits below always end);
//  2. wave 0 waits until every non-empty predecessor (offsets in {0,-1}^(D+1))
//     has signalled, bounded by the watchdog;
//  3. acquire (each wave), run `exec(P, k)`, release (each wave: the barrier
//     does not wait for outstanding stores), then one thread signals every
//     successor.
// Control values live in SGPRs (uni): with per-lane copies the compiler
// builds per-lane loops around the thread-0 regions that never terminate.
// DEVCOH: every global access of `exec` to tile data is device-coherent
// (buffer accesses with the SC1 policy), so acquiring needs no cache
// invalidation and releasing needs only the wait for store acknowledgements;
// otherwise agent-scope fences (L2 invalidate / write-back) are used.
template <int D, bool DEVCOH = false, typename Exec>
__device__ __forceinline__ void run_queued_tile(const TiledLaunch& Lc, int* s_tk, int* s_go, Exec&& exec) {
    const int wave = uni((int)(threadIdx.x >> 6));
    if (threadIdx.x == 0)
        *s_tk = (int)__hip_atomic_fetch_add(Lc.hdr + HDR_TICKET, 1u, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int tk = uni(*s_tk);
    if (tk >= Lc.nq) return;
    const QEntry e = Lc.queue[tk];
    const int pi = Lc.qprob ? uni((int)Lc.qprob[tk]) : 0;
    const TiledProblem P = Lc.probs[pi];
    int k[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) k[i] = uni((int)e.k[i]);
    unsigned* cnt = P.counters + tile_index(P, k, D);
    if (wave == 0) {
        unsigned need = 0;
#pragma unroll
        for (int m = 1; m < (1 << (D + 1)); ++m) {
            int q[4] = {0, 0, 0, 0};
#pragma unroll
            for (int i = 0; i <= D; ++i) q[i] = k[i] - ((m >> (D - i)) & 1);
            need += tile_nonempty<D>(P, q);
        }
        const bool go = wait_ready(cnt, need, Lc.hdr, Lc.limit_ticks);
        if (threadIdx.x == 0) *s_go = go ? 1 : 0;
    }
    __syncthreads();
    const int go = uni(*s_go);
    if constexpr (DEVCOH) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    else __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (go) exec(P, k);
    if constexpr (DEVCOH) {
        __builtin_amdgcn_s_waitcnt(0);  // every store of this wave acknowledged
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int m = 1; m < (1 << (D + 1)); ++m) {
            int q[4] = {0, 0, 0, 0};
            bool in = true;
#pragma unroll
            for (int i = 0; i <= D; ++i) {
                q[i] = k[i] + ((m >> (D - i)) & 1);
                in = in && q[i] < P.cnt[i];
            }
            if (in) signal(P.counters + tile_index(P, q, D));
        }
    }
}

// Pointer known to be the same in every lane, moved into SGPRs.
__device__ __forceinline__ const void* uptr(const void* p) {
    const uintptr_t v = (uintptr_t)p;
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
    return (const void*)(((uintptr_t)hi << 32) | lo);
}

// a if sel_b is even, b if odd, by bit masks (a conditional pick between
// two struct fields would be lowered to an indexed load from a stack copy).
__device__ __forceinline__ uintptr_t pick(uintptr_t a, uintptr_t b, int sel_b) {
    const uintptr_t m = (uintptr_t)0 - (uintptr_t)(sel_b & 1);
    return (a & ~m) | (b & m);
}

}  // namespace pcot
