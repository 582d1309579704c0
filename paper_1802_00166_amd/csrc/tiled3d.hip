// Time-skewed tile executor for the 7-point Heat-3D stencil.
//
// A leaf is t in [t0, t0+nt) x jz x jy x jx (skewed j = i + t, sizes bz, by,
// bx = 64).  Level t at (jz, jy, jx) updates u_{t+1} at (jz-t, jy-t, jx-t)
// from level t-1 outputs at
//   u  (jz-1, jy-1, jx-1),  x+ (jz-1, jy-1, jx),  x- (jz-1, jy-1, jx-2),
//   y+ (jz-1, jy,   jx-1),  y- (jz-1, jy-2, jx-1),
//   z+ (jz,   jy-1, jx-1),  z- (jz-2, jy-1, jx-1).
//
// Mapping: the block has by waves; thread (w, lane) owns column (jy0+w,
// jx0+lane).  Levels are pipelined along jz: at step s, level l handles plane
// jz0 + s - l, so the levels of one step are independent and one barrier per
// step suffices.  The input planes of every level but the first (outputs of
// the level below, with a two-wide halo in y and x holding the neighbour
// tiles' values) sit in a 4-slot LDS ring: plane jz being written, jz-1..jz-3
// readable.  Ring 0 holds the tile's input u_t0, streamed in plane by plane.
// The top level's outputs feed no level of the tile and go to memory only.
// Ring-0 planes and halos come from tiles that finished before this one
// started, so they are prefetched D steps ahead: a step is far shorter than
// a round trip to HBM.  For the common b_t the level count of a full tile is
// a compile-time constant: every step then runs every level (inactive ones,
// in the pipeline's fill and drain, skip their LDS write and store through
// an out-of-range offset), so each step issues the same memory instructions
// and the compiler's waits for a prefetch count exactly instead of covering
// every store in flight.  The planes below the tile (z-face) come from the
// z-neighbour tile at tile start.  Stores: the top level at every point, and
// the two-wide high faces in x, y and z of every other level.  Points outside
// the interior are carried unchanged.
#include "bufio.hpp"
#include "common.hpp"
#include "kernels.hpp"

#include <type_traits>

// Steps between a prefetch and its use (1, 2 or 4: the step loop is unrolled
// by four and a prefetch slot is the step it serves, mod the depth).
#ifndef PCOT_H3D_PREFETCH
#define PCOT_H3D_PREFETCH 2
#endif

namespace pcot {

namespace {

// Ring storage: the arithmetic type, except for bf16 storage, whose rings
// hold the 16-bit patterns.  Every value a bf16 ring receives is already a
// bf16 number (inputs read from bf16 storage, outputs rounded to bf16 by the
// update), so keeping its upper 16 bits is exact and halves the LDS a level
// needs.
template <typename S> struct Ring {
    using L = typename Tr<S>::A;
    static __device__ __forceinline__ L put(typename Tr<S>::A v) { return v; }
    static __device__ __forceinline__ typename Tr<S>::A get(L v) { return v; }
};
template <> struct Ring<uint16_t> {
    using L = uint16_t;
    static __device__ __forceinline__ L put(float v) { return (uint16_t)(__float_as_uint(v) >> 16); }
    static __device__ __forceinline__ float get(L v) { return bf16_to_f32(v); }
};

template <typename S, int BY, int D, bool BND, int NTC>
__device__ __forceinline__ void exec3d(const TiledProblem& P, const int* k, typename Ring<S>::L* lds) {
    using A = typename Tr<S>::A;
    using L = typename Ring<S>::L;
    using RG = Ring<S>;
    constexpr int ES = sizeof(S);
    constexpr int BX = 64, RX = BX + 2;
    const int lane = threadIdx.x & 63;
    const int w = uni((int)(threadIdx.x >> 6));
    constexpr int nthr = 64 * BY;
    const int nz = P.n[0], ny = P.n[1], nx = P.n[2];
    const int bt = P.b[0], bz = P.b[1];
    constexpr int by = BY;
    constexpr int RY = by + 2, PL = RY * RX;  // plane of the ring, with halo
    const int t0 = k[0] * bt;
    const int nt = NTC > 0 ? NTC : min(bt, P.T - t0);
    const int ttop = t0 + nt - 1;
    const int jz0 = 1 + k[1] * bz, jy0 = 1 + k[2] * by, jx0 = 1 + k[3] * BX;
    const uint32_t bytes = (uint32_t)nz * (uint32_t)ny * (uint32_t)nx * ES;
    const uintptr_t pin = (uintptr_t)uptr(P.in), pb0 = (uintptr_t)uptr(P.buf0), pb1 = (uintptr_t)uptr(P.buf1);
    auto src_of = [&](int t) {  // holds u_t
        return make_rsrc(uptr((const void*)pick(pick(pb0, pb1, t), pin, t == 0)), bytes);
    };
    auto inside = [&](int z, int y, int x) {
        return z >= 1 && z <= nz - 2 && y >= 1 && y <= ny - 2 && x >= 1 && x <= nx - 2;
    };
    auto offs = [&](int z, int y, int x) { return ((z * ny + y) * nx + x) * ES; };
    // ring v (v = 0: u_t0; v = l+1: outputs of level t0+l), plane jz, ring
    // row/col.  A plane's slot is the step that writes it, mod 4 (level l
    // writes plane jz0 + s - l of ring l+1 at step s; ring 0's plane jz0+s+1
    // is published at step s), so at step s every level reads slots s-1, s-2,
    // s-3 and writes slot s: with the step loop unrolled by four, all ring
    // addresses of a level are one base plus constants.
    auto ring = [&](int v, int jz, int ry, int rx) -> L& {
        return lds[((v * 4 + ((jz - jz0 + v + 3) & 3)) * RY + ry) * RX + rx];
    };

    static_assert(D == 1 || D == 2 || D == 4, "prefetch depth divides the unroll");
    // ---- tile start: planes jz0-2, jz0-1 of every ring, and plane jz0 of
    // ring 0; all loads of a ring are issued before its LDS stores, so a ring
    // costs one round trip to memory
    constexpr int TS = (3 * PL + nthr - 1) / nthr;
    for (int v = 0; v < nt; ++v) {
        const int np = v == 0 ? 3 : 2;
        const int d = t0 + v - 1;  // ring v holds u_{t0+v} at (j - d)
        const rsrc_t rs = src_of(t0 + v);
        A tv[TS];
#pragma unroll
        for (int i = 0; i < TS; ++i) {
            const int e = threadIdx.x + i * nthr;
            const int pz = e / PL, rem = e % PL;
            const int z = jz0 - 2 + pz - d, y = jy0 - 2 + rem / RX - d, x = jx0 - 2 + rem % RX - d;
            const bool ok = e < np * PL && z >= 0 && z < nz && y >= 0 && y < ny;
            tv[i] = IO<S>::ld(rs, ok ? offs(z, y, x) : OOB);
        }
#pragma unroll
        for (int i = 0; i < TS; ++i) {
            const int e = threadIdx.x + i * nthr;
            if (e < np * PL) {
                const int rem = e % PL;
                ring(v, jz0 - 2 + e / PL, rem / RX, rem % RX) = RG::put(tv[i]);
            }
        }
    }
    // Prefetch slots: every thread owns fixed positions of the ring-0 plane
    // and of the halos.  Their byte offsets and the steps in which they are
    // live are computed once per tile; a step then costs one add and two
    // unsigned compares per slot (32-bit multiplies are multi-pass on CDNA).
    const uint32_t PB = (uint32_t)ny * (uint32_t)nx * ES;  // bytes per plane
    constexpr int PF = (PL + nthr - 1) / nthr;             // ring-0 plane slots
    A p0[D][PF];
    int p_lds[PF];        // in-plane LDS index, -1: idle
    uint32_t p_off[PF];   // byte offset at step 0 (mod 2^32)
    bool p_yok[PF];       // slot in use and row inside the array
    const int d0 = t0 - 1;  // ring 0 holds u_t0 at (j - d0)
    // pf0_load(jz0 + s + 2) reads plane z = jz0 + s + 2 - d0: live while 0 <= z < nz
    const int zc0 = jz0 + 2 - d0;
#pragma unroll
    for (int i = 0; i < PF; ++i) {
        const int e = threadIdx.x + i * nthr;
        const int pr = e / RX, pc = e % RX;
        const int y = jy0 - 2 + pr - d0, x = jx0 - 2 + pc - d0;
        p_lds[i] = e < PL ? e : -1;
        p_yok[i] = e < PL && y >= 0 && y < ny;
        p_off[i] = (uint32_t)zc0 * PB + (uint32_t)(y * nx + x) * (uint32_t)ES;
    }
    // Every prefetch load is issued, with an out-of-range offset where
    // nothing is wanted, so that each step issues the same memory
    // instructions without branches and the compiler's waits count exactly
    // (a load skipped on some path makes it wait for every access in flight).
    const rsrc_t r0 = src_of(t0);
    auto pf0_load = [&](A (&dst)[PF], int s, bool live) {  // ring-0 plane jz0 + s + 2
        // the wave-uniform plane condition as an opaque VGPR mask OR-ed into
        // the offsets (a select on it is turned into a branch)
        uint32_t zm = (live && (uint32_t)(zc0 + s) < (uint32_t)nz) ? 0u : (uint32_t)OOB;
        asm volatile("" : "+v"(zm));
#pragma unroll
        for (int i = 0; i < PF; ++i)
            dst[i] = IO<S>::ld(r0, (int)((p_yok[i] ? p_off[i] + (uint32_t)s * PB : (uint32_t)OOB) | zm));
    };
    auto pf0_store = [&](const A (&src)[PF], int jz) {
        L* pl = &ring(0, jz, 0, 0);
#pragma unroll
        for (int i = 0; i < PF; ++i)
            if (p_lds[i] >= 0) pl[p_lds[i]] = RG::put(src[i]);
    };
    // halo of plane jz of ring v (1 <= v < nt): rows ry = 0, 1 (all RX
    // columns) and columns rx = 0, 1 of rows 2..RY-1: 2*RX + 2*by values per
    // level whose outputs are read in the tile (all but the top one)
    constexpr int HL = 2 * RX + 2 * by;
    constexpr int HPF = BY == 16 ? 2 : (BY == 8 ? 4 : 8);  // halo slots per thread per step (all levels)
    // both parity candidates of every halo value stay in registers until the
    // slot is published: selecting right after the loads would wait for them
    A hvE[D][HPF], hvO[D][HPF];
    // level (nt: idle), in-plane LDS index, first step with z >= 0 (far
    // below any step when the row lies outside the array), offset at step 0
    int h_l[HPF], h_lds[HPF], h_zlo[HPF];
    uint32_t h_off[HPF];
#pragma unroll
    for (int i = 0; i < HPF; ++i) {
        const int e = threadIdx.x + i * nthr;
        const int l = min(e / HL, nt), q = e % HL;
        int ry, rx;
        if (q < 2 * RX) { ry = q / RX; rx = q % RX; }
        else { ry = 2 + (q - 2 * RX) / 2; rx = (q - 2 * RX) & 1; }
        const int d = t0 + l;  // ring l+1 holds u_{t0+l+1} at (j - d)
        const int y = jy0 - 2 + ry - d, x = jx0 - 2 + rx - d;
        // at step s level l writes plane jz = jz0 + s - l, read at z = jz - d
        const int zc = jz0 - l - d;
        h_l[i] = l;
        h_lds[i] = ry * RX + rx;
        h_zlo[i] = (y >= 0 && y < ny) ? -zc : -(1 << 30);
        h_off[i] = (uint32_t)zc * PB + (uint32_t)(y * nx + x) * (uint32_t)ES;
    }
    // The lanes of one wave fetch halos of different levels, whose buffers
    // differ with the parity of t; a buffer descriptor must be wave-uniform,
    // so both are read (the other offset out of range) and the lane keeps its own.
    const rsrc_t rhE = src_of(t0 + 1), rhO = src_of(t0 + 2);  // rings v = l+1, l even / odd
    auto halo_load = [&](A (&dE)[HPF], A (&dO)[HPF], int s) {  // halos of the planes the levels write at step s
#pragma unroll
        for (int i = 0; i < HPF; ++i) {
            const int l = h_l[i];
            const bool ok = l + 1 < nt && (uint32_t)(s - l) < (uint32_t)bz && (uint32_t)(s - h_zlo[i]) < (uint32_t)nz;
            const int o = ok ? (int)(h_off[i] + (uint32_t)s * PB) : OOB;
            const bool ev = (l & 1) == 0;
            dE[i] = IO<S>::ld(rhE, ev ? o : OOB);
            dO[i] = IO<S>::ld(rhO, ev ? OOB : o);
        }
    };
    auto halo_store = [&](const A (&sE)[HPF], const A (&sO)[HPF], int s) {
#pragma unroll
        for (int i = 0; i < HPF; ++i) {
            const int l = h_l[i], sl = s - l;
            if (l + 1 < nt && (uint32_t)sl < (uint32_t)bz)
                (&ring(l + 1, jz0 + sl, 0, 0))[h_lds[i]] = RG::put((l & 1) ? sO[i] : sE[i]);
        }
    };
    // the data published at step q: ring-0 plane jz0 + q + 1 (level 0 reads
    // planes up to jz0 + bz - 1) and the halos of the planes written at step
    // q; slot q mod D
    auto fetch = [&](auto dc, int q) {
        constexpr int d = decltype(dc)::value;
        pf0_load(p0[d], q - 1, q <= bz - 2);
        halo_load(hvE[d], hvO[d], q);
    };
    // ring 0's slot is written at every step (past the tile's last plane
    // with values nobody reads): the plane it held was last read the step
    // before, and a load whose value were dropped on some path would again
    // cost a full wait
    auto publish = [&](auto dc, int q) {
        constexpr int d = decltype(dc)::value;
        pf0_store(p0[d], jz0 + q + 1);
        halo_store(hvE[d], hvO[d], q);
    };
    // On the generic path the level loop's trip count is known only at run
    // time, so the compiler cannot count the face stores it issues and a wait
    // for a prefetch also waits for every store issued since.  f64: the step's
    // prefetch goes after its stores, so such a wait covers only accesses at
    // least a step old (+8% on the generic path; for f32 and bf16 it measured
    // 5% slower or no different).
    constexpr bool FETCH_AFTER = sizeof(S) == 8;
    // steps padded to the unroll (the extra steps have no live level), so no
    // step is skipped by a branch
    const int nsteps = (bz + nt - 1 + 3) & ~3;
    fetch(std::integral_constant<int, 0>{}, 0);
    if constexpr (D > 1) fetch(std::integral_constant<int, 1>{}, 1);
    if constexpr (D > 2) {
        fetch(std::integral_constant<int, 2>{}, 2);
        fetch(std::integral_constant<int, 3>{}, 3);
    }
    __syncthreads();

    const int jy = jy0 + w, jx = jx0 + lane;
    const int ry = w + 2, rx = lane + 2;
    const int tc = (ry - 1) * RX + (rx - 1);  // the thread's centre input within a plane
    auto step = [&](auto qc, int s) {
        // slots of this step (s % 4 = Q): written, z+ plane, centre plane, z- plane
        constexpr int Q = decltype(qc)::value;
        constexpr int SW = Q, SP = (Q + 3) & 3, SC = (Q + 2) & 3, SM = (Q + 1) & 3;
        // publish the prefetched ring-0 plane jz0+s+1 and the halos of this
        // step's output planes, then refill the slot for step s + D
        publish(std::integral_constant<int, Q % D>{}, s);
        __syncthreads();
        if constexpr (!FETCH_AFTER) fetch(std::integral_constant<int, Q % D>{}, s + D);
        if constexpr (NTC > 0) {
            // every level of a full tile, active or not
#pragma unroll
            for (int l = 0; l < NTC; ++l) {
                const int jz = jz0 + s - l;
                const bool act = jz >= jz0 && jz < jz0 + bz;  // uniform
                const int t = t0 + l;
                const L* rl = lds + l * (4 * PL) + tc;
                const A u = RG::get(rl[SC * PL]);
                const A v = Tr<S>::rnd(heat3(u, RG::get(rl[SC * PL + 1]), RG::get(rl[SC * PL - 1]),
                                             RG::get(rl[SC * PL + RX]), RG::get(rl[SC * PL - RX]),
                                             RG::get(rl[SP * PL]), RG::get(rl[SM * PL])));
                const int z = jz - t, y = jy - t, x = jx - t;
                const bool in = !BND || inside(z, y, x);
                const A out = in ? v : u;
                if (l + 1 < NTC && act) lds[(l + 1) * (4 * PL) + SW * PL + ry * RX + rx] = RG::put(out);
                const bool face = t == ttop || lane >= BX - 2 || w >= by - 2 || jz >= jz0 + bz - 2;
                IO<S>::st((l & 1) ? rhO : rhE, (act && face && in) ? offs(z, y, x) : OOB, out);
            }
        } else
        for (int l = 0; l < nt; ++l) {
            const int jz = jz0 + s - l;
            if (jz < jz0 || jz >= jz0 + bz) continue;  // uniform
            const int t = t0 + l;
            const L* rl = lds + l * (4 * PL) + tc;  // ring l around the centre input
            const A u = RG::get(rl[SC * PL]);
            const A v = Tr<S>::rnd(heat3(u, RG::get(rl[SC * PL + 1]), RG::get(rl[SC * PL - 1]),
                                         RG::get(rl[SC * PL + RX]), RG::get(rl[SC * PL - RX]),
                                         RG::get(rl[SP * PL]), RG::get(rl[SM * PL])));
            const int z = jz - t, y = jy - t, x = jx - t;
            const bool in = !BND || inside(z, y, x);
            const A out = in ? v : u;
            if (l + 1 < nt) lds[(l + 1) * (4 * PL) + SW * PL + ry * RX + rx] = RG::put(out);
            const bool face = t == ttop || lane >= BX - 2 || w >= by - 2 || jz >= jz0 + bz - 2;
            // level l writes u_{t0+l+1}: the buffers of rings l+1 (hoisted descriptors)
            if (face && in) IO<S>::st((l & 1) ? rhO : rhE, offs(z, y, x), out);
        }
        if constexpr (FETCH_AFTER) fetch(std::integral_constant<int, Q % D>{}, s + D);
        __syncthreads();
    };
    for (int s0 = 0; s0 < nsteps; s0 += 4) {
        step(std::integral_constant<int, 0>{}, s0);
        step(std::integral_constant<int, 1>{}, s0 + 1);
        step(std::integral_constant<int, 2>{}, s0 + 2);
        step(std::integral_constant<int, 3>{}, s0 + 3);
    }
}

template <typename S, int BY, int BT>
__global__ void __launch_bounds__(64 * BY) k_tiled3d(TiledLaunch Lc) {
    extern __shared__ char smem_raw[];
    using L = typename Ring<S>::L;
    __shared__ int s_tk, s_go;
    run_queued_tile<3, true>(Lc, &s_tk, &s_go, [&](const TiledProblem& P, const int* k) {
        // tiles whose every point lies inside the array skip the per-point test
        const bool full = BT > 0 && P.b[0] == BT && (k[0] + 1) * BT <= P.T;
        if (full) {
            if (tile_interior<3>(P, k))
                exec3d<S, BY, PCOT_H3D_PREFETCH, false, BT>(P, k, reinterpret_cast<L*>(smem_raw));
            else
                exec3d<S, BY, PCOT_H3D_PREFETCH, true, BT>(P, k, reinterpret_cast<L*>(smem_raw));
        } else if (tile_interior<3>(P, k)) {
            exec3d<S, BY, PCOT_H3D_PREFETCH, false, 0>(P, k, reinterpret_cast<L*>(smem_raw));
        } else {
            exec3d<S, BY, PCOT_H3D_PREFETCH, true, 0>(P, k, reinterpret_cast<L*>(smem_raw));
        }
    });
}

template <typename S, int BY, int BT>
hipError_t launch_bt(const TiledLaunch& Lc, size_t lds, hipStream_t s) {
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute((const void*)k_tiled3d<S, BY, BT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_tiled3d<S, BY, BT>), dim3(Lc.nq), dim3(64 * BY), lds, s, Lc);
    return hipGetLastError();
}

// b_t with a kernel of its own (its full tiles take the fixed-level path);
// other b_t run every tile on the generic path
template <typename S, int BY>
hipError_t launch_by(const TiledLaunch& Lc, int bt, size_t lds, hipStream_t s) {
    switch (bt) {
        case 2: return launch_bt<S, BY, 2>(Lc, lds, s);
        case 3: return launch_bt<S, BY, 3>(Lc, lds, s);
        case 4: return launch_bt<S, BY, 4>(Lc, lds, s);
        case 6: return launch_bt<S, BY, 6>(Lc, lds, s);
        case 8: return launch_bt<S, BY, 8>(Lc, lds, s);
        case 12: return launch_bt<S, BY, 12>(Lc, lds, s);
        default: return launch_bt<S, BY, 0>(Lc, lds, s);
    }
}

template <typename S>
hipError_t launch_dtype(const int* b, const TiledLaunch& Lc, hipStream_t s) {
    if (Lc.nq <= 0) return hipSuccess;
    const int bt = b[0], by = b[2];
    const size_t lds = (size_t)bt * 4 * (by + 2) * 66 * sizeof(typename Ring<S>::L);
    switch (by) {
        case 2: return launch_by<S, 2>(Lc, bt, lds, s);
        case 4: return launch_by<S, 4>(Lc, bt, lds, s);
        case 8: return launch_by<S, 8>(Lc, bt, lds, s);
        case 16: return launch_by<S, 16>(Lc, bt, lds, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool tiled3d_supported(const int* b, int lds_elem) {
    // b = {bt, bz, by, bx}; lds_elem: bytes of one ring value (8 f64, 4 f32, 2 bf16)
    if (b[3] != 64) return false;
    if (b[2] != 2 && b[2] != 4 && b[2] != 8 && b[2] != 16) return false;
    if (b[1] < 2 || b[0] < 1 || b[0] > 16) return false;
    // halo prefetch slots: HPF * threads >= (bt - 1) * (2*66 + 2*by)
    const int hpf = b[2] == 16 ? 2 : (b[2] == 8 ? 4 : 8);
    if (hpf * 64 * b[2] < (b[0] - 1) * (2 * 66 + 2 * b[2])) return false;
    // rings: the tile's input and the outputs of every level but the top one
    const size_t lds = (size_t)b[0] * 4 * (b[2] + 2) * 66 * lds_elem;
    return lds <= 150 * 1024;
}

hipError_t launch_tiled3d(int dtype, const int* b, const TiledLaunch& Lc, int, hipStream_t s) {
    switch (dtype) {
        case 0: return launch_dtype<double>(b, Lc, s);
        case 1: return launch_dtype<float>(b, Lc, s);
        default: return launch_dtype<uint16_t>(b, Lc, s);
    }
}

}  // namespace pcot
