// Executor of the concurrent-start trapezoid schedules for the 5-point
// Jacobi-2D stencil (tile geometry and phases: trap.hpp).
//
// A block of G waves holds a tile's footprint, FY = G*R rows by FX = 64*C
// columns with a one-point halo, in registers for the whole band: wave w owns
// footprint rows [w*R, w*R + R), lane owns columns [lane*C, lane*C + C).
// Level by level the block updates every row of the level's row range in
// place (one row of old values kept for the north neighbour), taking east
// and west neighbours across lanes with DPP shifts and the rows above and
// below the wave from its neighbour waves through LDS (one barrier per
// level).  Columns outside the level's column range are computed too and
// never stored: a growing side reloads the two columns it needs next from
// the tile beside it before every level, so these values are never used.
//
// Global traffic per tile: the level-0 range plus halo at the start; before
// each level the two-wide faces of the growing sides (written by the
// neighbouring tiles at the previous level); after each level the two
// outermost rows / columns of the shrinking sides; the top level at the end.
// All of it goes through buffer resources with the device-coherent (SC1)
// policy, so a tile only waits for its stores to be acknowledged before it
// signals its successors.  Blocks are persistent: each takes tiles from the
// queue by ticket until the queue is empty; every predecessor of a ticket is
// held by a running block or done, so every wait ends.
#include "bufio.hpp"
#include "common.hpp"
#include "trap.hpp"

#include <algorithm>
#include <type_traits>

// (band height, footprint rows, footprint columns) of the compiled executors
#define PCOT_TRAP_INSTANCES(X) X(16, 64, 128) X(8, 64, 128) X(8, 32, 128)

namespace pcot {

namespace {

// Value of lane+1 (DPP wave_shl:1); lane 63 receives `fill`.
__device__ __forceinline__ float shl1(float v, float fill) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(fill), __float_as_int(v),
                                                      0x130, 0xF, 0xF, false));
}
__device__ __forceinline__ double shl1(double v, double fill) {
    const long long vi = __double_as_longlong(v), fi = __double_as_longlong(fill);
    const int lo = __builtin_amdgcn_update_dpp((int)fi, (int)vi, 0x130, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(fi >> 32), (int)(vi >> 32), 0x130, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// C consecutive elements of one lane: loaded and stored in 16-byte pieces.
template <typename S, int C> struct VecIO;
template <int C> struct VecIO<double, C> {
    static_assert(C % 2 == 0, "f64 tiles hold an even number of columns per lane");
    static __device__ __forceinline__ void ld(rsrc_t r, int off, double (&v)[C]) {
#pragma unroll
        for (int i = 0; i < C; i += 2) {
            const u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(r, off + i * 8, 0, CPOL_DEV);
            v[i] = __builtin_bit_cast(double, u32x2{q.x, q.y});
            v[i + 1] = __builtin_bit_cast(double, u32x2{q.z, q.w});
        }
    }
    static __device__ __forceinline__ void st(rsrc_t r, int off, const double (&v)[C]) {
#pragma unroll
        for (int i = 0; i < C; i += 2) {
            const u32x2 a = __builtin_bit_cast(u32x2, v[i]), b = __builtin_bit_cast(u32x2, v[i + 1]);
            __builtin_amdgcn_raw_buffer_store_b128(u32x4{a.x, a.y, b.x, b.y}, r, off + i * 8, 0, CPOL_DEV);
        }
    }
};
template <int C> struct VecIO<float, C> {
    static_assert(C % 2 == 0, "f32 tiles hold an even number of columns per lane");
    static __device__ __forceinline__ void ld(rsrc_t r, int off, float (&v)[C]) {
#pragma unroll
        for (int i = 0; i < C; i += 2) {
            const u32x2 q = __builtin_amdgcn_raw_buffer_load_b64(r, off + i * 4, 0, CPOL_DEV);
            v[i] = __uint_as_float(q.x);
            v[i + 1] = __uint_as_float(q.y);
        }
    }
    static __device__ __forceinline__ void st(rsrc_t r, int off, const float (&v)[C]) {
#pragma unroll
        for (int i = 0; i < C; i += 2)
            __builtin_amdgcn_raw_buffer_store_b64(u32x2{__float_as_uint(v[i]), __float_as_uint(v[i + 1])}, r,
                                                  off + i * 4, 0, CPOL_DEV);
    }
};

template <typename A, int C, int G, int R, int BT> struct TrapSmem {
    A yf[BT][2][2][64 * C];  // y faces by level: [level][low, high side][row pair][column]
    A xf[BT][2][G * R][2];   // x faces by level: [level][low, high side][row][column pair]
    A xch[2][G][2][64 * C];  // [level parity][wave][first, last row][column]
    int tk, go;
};

template <int I, int N, typename F> __device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// One tile: footprint in registers, levels unrolled (nt <= BT of them run).
// Global -> LDS copy without registers (one dword per lane, LDS destination
// base + 4 * lane, wave-uniform base); completion counts in vmcnt.
__device__ __forceinline__ void dma_dword(rsrc_t r, void* lds_base, int voff) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)lds_base, 4, voff, 0, 0,
                                             CPOL_DEV);
}

template <typename S, int C, int R, int G, int BT, bool BND>
__device__ __forceinline__ void trap_tile(const TrapLaunch& L, const TrapTile& t,
                                          TrapSmem<typename Tr<S>::A, C, G, R, BT>& sm) {
    using A = typename Tr<S>::A;
    constexpr int ES = sizeof(S), FY = G * R, FX = 64 * C;
    const int lane = threadIdx.x & 63;
    const int w = uni((int)(threadIdx.x >> 6));
    const int ny = L.ny, nx = L.nx;
    const int fy0 = t.fo[0], fx0 = t.fo[1];
    const int ry0 = fy0 + w * R;     // array row of the wave's first row
    const int cx0 = fx0 + lane * C;  // array column of the lane's first column
    const uint32_t bytes = (uint32_t)ny * (uint32_t)nx * ES;
    const uintptr_t pin = (uintptr_t)uptr(L.in), pb0 = (uintptr_t)uptr(L.buf0), pb1 = (uintptr_t)uptr(L.buf1);
    auto src_of = [&](int tt) {  // holds u_tt
        return make_rsrc(uptr((const void*)pick(pick(pb0, pb1, tt), pin, tt == 0)), bytes);
    };
    auto dst_of = [&](int tt) {  // receives u_{tt+1}
        return make_rsrc(uptr((const void*)pick(pb0, pb1, tt + 1)), bytes);
    };
    auto yrange = [&](int l, int& a, int& b) {
        a = max(t.lo[0] + t.slo[0] * l, 1);
        b = min(t.hi[0] + t.shi[0] * l, ny - 1);
    };
    auto xrange = [&](int l, int& a, int& b) {
        a = max(t.lo[1] + t.slo[1] * l, 1);
        b = min(t.hi[1] + t.shi[1] * l, nx - 1);
    };
    auto lane_meets = [&](int a, int b) { return cx0 + C > a && cx0 < b && a < b; };
    unsigned colin = (1u << C) - 1u;  // BND: bit c = column c of the lane is interior
    if (BND) {
        colin = 0;
#pragma unroll
        for (int c = 0; c < C; ++c) colin |= (cx0 + c >= 1 && cx0 + c <= nx - 2) ? (1u << c) : 0u;
    }
    // one row segment [a, b) of a lane's columns to global memory: whole
    // vectors where the lane lies inside, single elements at the ends
    auto store_row = [&](rsrc_t rd, int y, int a, int b, const A (&v)[C]) {
        const int off = (y * nx + cx0) * ES;
        const bool full = cx0 >= a && cx0 + C <= b;
        VecIO<S, C>::st(rd, full ? off : OOB, v);
        if (uni((int)((((a - fx0) % C) != 0) || (((b - fx0) % C) != 0)))) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const bool ok = !full && cx0 + c >= a && cx0 + c < b;
                IO<S>::st(rd, ok ? off + c * ES : OOB, v[c]);
            }
        }
    };

    // Every face of every level is final when the tile starts (its producers
    // are predecessors), so all of them are copied to LDS up front with
    // register-free DMA loads, beside the level-0 loads: one memory round
    // trip per tile instead of one per level.  A V side of natural start b
    // sits at footprint index BT (low) or F - BT (high); level l needs the
    // two points just outside the range it had at level l-1.
    {
        constexpr int RW = 64 * C * ES / 4;  // dwords per footprint row
        const int nl = t.nt;
        const bool ylo = t.slo[0] < 0, yhi = t.shi[0] > 0, xlo = t.slo[1] < 0, xhi = t.shi[1] > 0;
        // y faces: (level, side, row of pair, 256-byte piece) jobs, dealt to waves
        const int ny_jobs = (nl - 1) * 2 * 2 * (RW / 64);
        for (int j = w; j < ny_jobs; j += G) {
            const int piece = j % (RW / 64), k = (j / (RW / 64)) % 2, sd = (j / (RW / 64) / 2) % 2;
            const int l = 1 + j / (RW / 64) / 4;
            if (!(sd ? yhi : ylo)) continue;
            const int f = sd ? FY - BT + l - 1 + k : BT - l - 1 + k;
            const rsrc_t rs = src_of(t.t0 + l);
            const int voff = ((fy0 + f) * nx + fx0) * ES + (piece * 64 + lane) * 4;
            dma_dword(rs, (char*)&sm.yf[l][sd][k][0] + piece * 256, (f >= 0 && f < FY) ? voff : OOB);
        }
        // x faces: (level, side, 16-row piece) jobs; lane -> (row, dword of the pair)
        constexpr int XD = 2 * ES / 4;  // dwords per row of a column pair
        constexpr int XR = 64 / XD;     // rows per DMA instruction
        const int nx_jobs = (nl - 1) * 2 * (FY / XR);
        for (int j = w; j < nx_jobs; j += G) {
            const int piece = j % (FY / XR), sd = (j / (FY / XR)) % 2, l = 1 + j / (FY / XR) / 2;
            if (!(sd ? xhi : xlo)) continue;
            const int f = sd ? FX - BT + l - 1 : BT - l - 1;
            const int row = piece * XR + lane / XD;
            const rsrc_t rs = src_of(t.t0 + l);
            const int voff = ((fy0 + row) * nx + fx0 + f) * ES + (lane % XD) * 4;
            dma_dword(rs, (char*)&sm.xf[l][sd][piece * XR][0], voff);
        }
    }
    A H[R][C];
    {  // level-0 inputs: u_t0 over the level-0 range plus halo
        int ya, yb, xa, xb;
        yrange(0, ya, yb);
        xrange(0, xa, xb);
        const rsrc_t rs = src_of(t.t0);
        const bool lok = lane_meets(xa - 1, xb + 1);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int y = ry0 + r;
            if (y >= ya - 1 && y < yb + 1) VecIO<S, C>::ld(rs, lok ? (y * nx + cx0) * ES : OOB, H[r]);
        }
    }
    __builtin_amdgcn_s_waitcnt(0);  // DMA data in LDS, level-0 rows in registers
    __syncthreads();

    static_for<0, BT>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        if (l >= t.nt) return;
        int ya, yb, xa, xb;
        yrange(l, ya, yb);
        xrange(l, xa, xb);
        if constexpr (l > 0) {
            // faces of the growing sides (u_{t0+l}, from the LDS copies)
            auto face_row = [&](auto fc, int sd, int k) {
                constexpr int f = decltype(fc)::value;
                if constexpr (f >= 0 && f < FY) {
                    if (w == f / R) {
#pragma unroll
                        for (int c = 0; c < C; ++c) H[f % R][c] = sm.yf[l][sd][k][lane * C + c];
                    }
                }
            };
            auto face_col = [&](auto fc, int sd, int k) {
                constexpr int f = decltype(fc)::value;
                if constexpr (f >= 0 && f < FX) {
                    const bool mine = lane == f / C;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const A v = sm.xf[l][sd][w * R + r][k];
                        H[r][f % C] = mine ? v : H[r][f % C];
                    }
                }
            };
            using std::integral_constant;
            if (t.slo[0] < 0) {
                face_row(integral_constant<int, BT - l - 1>{}, 0, 0);
                face_row(integral_constant<int, BT - l>{}, 0, 1);
            }
            if (t.shi[0] > 0) {
                face_row(integral_constant<int, FY - BT + l - 1>{}, 1, 0);
                face_row(integral_constant<int, FY - BT + l>{}, 1, 1);
            }
            if (t.slo[1] < 0) {
                face_col(integral_constant<int, BT - l - 1>{}, 0, 0);
                face_col(integral_constant<int, BT - l>{}, 0, 1);
            }
            if (t.shi[1] > 0) {
                face_col(integral_constant<int, FX - BT + l - 1>{}, 1, 0);
                face_col(integral_constant<int, FX - BT + l>{}, 1, 1);
            }
        }
        // rows next to the wave (level l-1 values) from the neighbour waves
        A* xw = &sm.xch[l & 1][w][0][0];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            xw[lane * C + c] = H[0][c];
            xw[64 * C + lane * C + c] = H[R - 1][c];
        }
        __syncthreads();
        A nb[C], sb[C];
        {
            const A* up = &sm.xch[l & 1][w > 0 ? w - 1 : 0][1][0];
            const A* dn = &sm.xch[l & 1][w + 1 < G ? w + 1 : G - 1][0][0];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                nb[c] = up[lane * C + c];
                sb[c] = dn[lane * C + c];
            }
        }
        // level l in place, row by row
        A prev[C];
#pragma unroll
        for (int c = 0; c < C; ++c) prev[c] = nb[c];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int y = ry0 + r;
            A old[C];
#pragma unroll
            for (int c = 0; c < C; ++c) old[c] = H[r][c];
            if (y >= ya && y < yb) {
                const A wv = shr1(old[C - 1], old[C - 1]);  // lane-1's last column
                const A ev = shl1(old[0], old[0]);          // lane+1's first column
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const A cc = old[c];
                    const A nn = prev[c];
                    const A ss = r + 1 < R ? H[r + 1 < R ? r + 1 : 0][c] : sb[c];
                    const A ee = c + 1 < C ? old[c + 1 < C ? c + 1 : 0] : ev;
                    const A ww = c > 0 ? old[c > 0 ? c - 1 : 0] : wv;
                    A v = Tr<S>::rnd(jac2(cc, nn, ss, ee, ww));
                    if (BND) v = ((colin >> c) & 1u) ? v : cc;
                    H[r][c] = v;
                }
            }
#pragma unroll
            for (int c = 0; c < C; ++c) prev[c] = old[c];
        }
        // stores of level l: u_{t0+l+1}
        const rsrc_t rd = dst_of(t.t0 + l);
        if (l == t.nt - 1) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int y = ry0 + r;
                if (y >= ya && y < yb) store_row(rd, y, xa, xb, H[r]);
            }
        } else {
            // the two outermost rows / columns of every shrinking side: the
            // tile beside it computes their neighbours at level l+1
            auto st_row = [&](auto fc) {
                constexpr int f = decltype(fc)::value;
                if constexpr (f >= 0 && f < FY) {
                    const int y = fy0 + f;
                    if (w == f / R && y >= ya && y < yb) store_row(rd, y, xa, xb, H[f % R]);
                }
            };
            auto st_col = [&](auto fc) {
                constexpr int f = decltype(fc)::value;
                if constexpr (f >= 0 && f < FX) {
                    const int x = fx0 + f;
                    if (x >= xa && x < xb) {
                        const bool mine = lane == f / C;
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const int y = ry0 + r;
                            if (y >= ya && y < yb) IO<S>::st(rd, mine ? (y * nx + x) * ES : OOB, H[r][f % C]);
                        }
                    }
                }
            };
            using std::integral_constant;
            if (t.slo[0] > 0) {
                st_row(integral_constant<int, 1 + l>{});
                st_row(integral_constant<int, 2 + l>{});
            }
            if (t.shi[0] < 0) {
                st_row(integral_constant<int, FY - 3 - l>{});
                st_row(integral_constant<int, FY - 2 - l>{});
            }
            if (t.slo[1] > 0) {
                st_col(integral_constant<int, 1 + l>{});
                st_col(integral_constant<int, 2 + l>{});
            }
            if (t.shi[1] < 0) {
                st_col(integral_constant<int, FX - 3 - l>{});
                st_col(integral_constant<int, FX - 2 - l>{});
            }
        }
    });
}

template <typename S, int C, int R, int G, int BT>
__global__ void __launch_bounds__(64 * G) k_trap2d(TrapLaunch L) {
    static_assert(G * R >= 2 * BT + 2 && 64 * C >= 2 * BT + 2, "footprint too small for the band height");
    using A = typename Tr<S>::A;
    __shared__ TrapSmem<A, C, G, R, BT> sm;
    constexpr int FX = 64 * C;
    for (;;) {
        if (threadIdx.x == 0)
            sm.tk = (int)__hip_atomic_fetch_add(L.hdr + HDR_TICKET, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int tk = uni(sm.tk);
        if (tk >= L.ntiles) return;
        const TrapTile t = L.tiles[tk];
        if (threadIdx.x < 64) {
            const bool go = wait_ready(L.counters + tk, (unsigned)t.need, L.hdr, L.limit_ticks);
            if (threadIdx.x == 0) sm.go = go ? 1 : 0;
        }
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (uni(sm.go)) {
            const bool bnd = t.fo[1] < 1 || t.fo[1] + FX > L.nx - 1;
            if (bnd) trap_tile<S, C, R, G, BT, true>(L, t, sm);
            else trap_tile<S, C, R, G, BT, false>(L, t, sm);
        }
        __builtin_amdgcn_s_waitcnt(0);  // every store of this wave acknowledged
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        if (threadIdx.x == 0)
            for (int i = 0; i < t.nsucc; ++i) signal(L.counters + L.succ[t.succ0 + i]);
    }
}

template <typename S, int C, int R, int G, int BT>
hipError_t launch_inst(const TrapLaunch& L, hipStream_t s) {
    static int grid = 0;  // resident blocks on the whole device (persistent grid)
    if (!grid) {
        int dev = 0, cus = 0, per = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_trap2d<S, C, R, G, BT>, 64 * G, 0);
        if (e != hipSuccess) return e;
        grid = std::max(1, cus * std::max(1, per));
    }
    const int nb = std::min(grid, L.ntiles);
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_trap2d<S, C, R, G, BT>), dim3(nb), dim3(64 * G), 0, s, L);
    return hipGetLastError();
}

// Instances: (bt, footprint rows, footprint columns); rows are 8 per wave.
template <typename S> hipError_t launch_dtype(int bt, int fy, int fx, const TrapLaunch& L, hipStream_t s) {
#define PCOT_TRAP_CASE(BT_, FY_, FX_)                                             \
    if (bt == BT_ && fy == FY_ && fx == FX_) return launch_inst<S, FX_ / 64, 8, FY_ / 8, BT_>(L, s);
    PCOT_TRAP_INSTANCES(PCOT_TRAP_CASE)
#undef PCOT_TRAP_CASE
    return hipErrorInvalidValue;
}

}  // namespace

bool trap2d_supported(int dtype, int bt, int fy, int fx) {
    if (dtype != 0) return false;
#define PCOT_TRAP_CASE(BT_, FY_, FX_) \
    if (bt == BT_ && fy == FY_ && fx == FX_) return true;
    PCOT_TRAP_INSTANCES(PCOT_TRAP_CASE)
#undef PCOT_TRAP_CASE
    return false;
}

hipError_t launch_trap2d(int dtype, int bt, int fy, int fx, const TrapLaunch& L, hipStream_t s) {
    if (dtype == 0) return launch_dtype<double>(bt, fy, fx, L, s);
    return hipErrorInvalidValue;
}

}  // namespace pcot
