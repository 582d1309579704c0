// C ABI: argument validation, plan cache, workspace layout and launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <array>
#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/pcot.h"
#include "kernels.hpp"
#include "plan.hpp"
#include "trap.hpp"
#include "front.hpp"
#include "motiv.hpp"
#include "dpsplit.hpp"
#include "resident.hpp"

namespace pcot {
enum : int { DP_INIT = 0, DP_ITEMS = 1, DP_FINISH = 2 };
struct DPLaunch {
    const long long* p;
    void* Cw;
    long long* C;
    int N, Nout, b;
    const int2* tiles;
    int ntiles;
    const int4* items;
    int nitems;
    unsigned* hdr;
    long long pmax;
};
bool dp_block_supported(int b);
hipError_t launch_dp_phase(bool wide, const DPLaunch& a, int mode, hipStream_t s);
hipError_t launch_dp_pad(const long long* p, long long* pp, int Nout, int N, hipStream_t s);
}  // namespace pcot

using namespace pcot;

namespace {
thread_local std::string g_err;
}  // namespace

// Records the message of a failing call (read back by pcot_last_error).
pcot_status pcot::fail(pcot_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

namespace {

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) return fail(PCOT_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t ALIGN = 256;
// First byte offset the tiled executors treat as out of range (the store
// mask offset of their buffer resources).
constexpr uint32_t TILED_MAX_OFFSET = 0x7FFFFFF0u;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

bool is_trap(int schedule) { return schedule == PCOT_TRAP || schedule == PCOT_DIAMOND; }

size_t elem_bytes(int dtype) { return dtype == PCOT_F64 ? 8 : dtype == PCOT_F32 ? 4 : 2; }

int kind_dims(int kind) {
    switch (kind) {
        case PCOT_JACOBI1D_3PT: case PCOT_MOTIV1D: return 1;
        case PCOT_JACOBI2D_5PT: case PCOT_GS2D_5PT: case PCOT_FDTD2D: return 2;
        case PCOT_HEAT3D_7PT: return 3;
        default: return 0;
    }
}

// Kinds updated in place by the front executor (dependences inside a step).
bool is_front(int kind) { return kind == PCOT_GS2D_5PT || kind == PCOT_FDTD2D; }
// Fields of a kind (FDTD-2D: ex, ey, hz one after another).
int kind_fields(int kind) { return kind == PCOT_FDTD2D ? 3 : 1; }

long long watchdog_ticks() {
    // wall_clock64 runs at hipDeviceAttributeWallClockRate kHz; allow 4 s.
    static long long ticks = 0;
    if (!ticks) {
        int dev = 0, khz = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
            khz = 100000;
        ticks = (long long)khz * 1000LL * 4LL;
    }
    return ticks;
}

// ------------------------------------------------------------- validation ---
struct Prob {
    int kind = 0, dtype = 0, d = 0, sched = 0;
    int64_t n[3] = {1, 1, 1};
    int64_t T = 0;
    int b[4] = {1, 1, 1, 1};   // t, spatial outer..inner
    int64_t elems = 0;
};

pcot_status validate(int32_t kind, int32_t dtype, const int64_t* dims, int64_t T, const pcot_tile* tile,
                     int32_t schedule, Prob& p) {
    p.kind = kind;
    p.dtype = dtype;
    p.d = kind_dims(kind);
    p.sched = schedule;
    if (!p.d) return fail(PCOT_ERR_INVALID, "unknown kind %d", kind);
    if (dtype < PCOT_F64 || dtype > PCOT_BF16) return fail(PCOT_ERR_INVALID, "unknown dtype %d", dtype);
    if (schedule < PCOT_NAIVE || schedule > PCOT_DIAMOND) return fail(PCOT_ERR_INVALID, "unknown schedule %d", schedule);
    if (is_trap(schedule) && kind != PCOT_JACOBI2D_5PT)
        return fail(PCOT_ERR_UNSUPPORTED, "trapezoid schedules are built for the Jacobi-2D stencil only");
    if ((is_front(kind) || kind == PCOT_MOTIV1D) && dtype != PCOT_F64)
        return fail(PCOT_ERR_UNSUPPORTED, "Gauss-Seidel-2D, FDTD-2D and the motivating 1D program run in f64 only");
    if (kind == PCOT_GS2D_5PT && schedule == PCOT_NAIVE)
        return fail(PCOT_ERR_UNSUPPORTED, "Gauss-Seidel-2D has no untiled executor (its sweep is sequential)");
    if (!dims) return fail(PCOT_ERR_INVALID, "dims is NULL");
    if (T < 0 || T > (1 << 30)) return fail(PCOT_ERR_INVALID, "T=%lld out of range", (long long)T);
    p.T = T;
    p.elems = 1;
    for (int i = 0; i < p.d; ++i) {
        const int64_t lo = kind == PCOT_FDTD2D ? 1 : 3;  // FDTD cells have no fixed frame
        if (dims[i] < lo || dims[i] > (1LL << 30))
            return fail(PCOT_ERR_INVALID, "dims[%d]=%lld (need %lld .. 2^30)", i, (long long)dims[i], (long long)lo);
        p.n[i] = dims[i];
        p.elems *= dims[i];
    }
    if (p.elems > (1LL << 36)) return fail(PCOT_ERR_INVALID, "field too large");
    if (schedule != PCOT_NAIVE) {
        if (!tile) return fail(PCOT_ERR_INVALID, "tile is NULL for a tiled schedule");
        if (tile->t < 1) return fail(PCOT_ERR_INVALID, "tile.t=%d < 1", tile->t);
        p.b[0] = tile->t;
        for (int i = 0; i < p.d; ++i) {
            if (tile->s[i] < 2) return fail(PCOT_ERR_INVALID, "tile.s[%d]=%d < 2 (dependence distance is 2)", i, tile->s[i]);
            p.b[i + 1] = tile->s[i];
        }
        if (is_trap(schedule)) {
            for (int i = 0; i < 2; ++i)
                if (tile->s[i] < 2 * tile->t + 2)
                    return fail(PCOT_ERR_INVALID, "trapezoid footprint s[%d]=%d < 2*t+2 = %d", i, tile->s[i],
                                2 * tile->t + 2);
            // the host plan lists every tile with its successors: bound its size
            double tiles = (double)((T + tile->t - 1) / tile->t);
            for (int i = 0; i < 2; ++i) {
                const double period = 2.0 * tile->s[i] - 2.0 - 2.0 * tile->t;
                tiles *= 2.0 * (std::ceil((double)dims[i] / period) + 1.0);
            }
            if (tiles > (double)(1 << 24))
                return fail(PCOT_ERR_UNSUPPORTED, "trapezoid plan of about %.0f tiles (limit 2^24): use a larger tile",
                            tiles);
        }
        // The tiled executors address a field through one buffer resource
        // with 32-bit byte offsets and mask stores with the offset OOB
        // (0x7FFFFFF0).  Offsets they form reach one outermost slice (row,
        // plane) past either end of the array, so the field plus two such
        // slices must stay below OOB.
        const int64_t es = (int64_t)elem_bytes(dtype);
        const int64_t slice = p.elems / p.n[0] * es;
        if (p.elems * es + 2 * slice + 4096 > (int64_t)TILED_MAX_OFFSET)
            return fail(PCOT_ERR_UNSUPPORTED,
                        "field of %lld bytes: the tiled executors need field + 2 outer slices + 4 KiB below %lld bytes",
                        (long long)(p.elems * es), (long long)TILED_MAX_OFFSET);
    }
    return PCOT_OK;
}

bool tile_ok(int kind, int dtype, const int* b, int schedule = PCOT_SLT_WAVE) {
    if (is_trap(schedule)) return kind == PCOT_JACOBI2D_5PT && trap2d_supported(dtype, b[0], b[1], b[2]);
    if (is_front(kind)) return front2d_supported(kind, dtype, b);
    if (kind == PCOT_MOTIV1D) return dtype == PCOT_F64 && motiv_supported(b);
    int bb[4] = {b[0], b[1], b[2], b[3]};
    switch (kind) {
        case PCOT_JACOBI1D_3PT: return tiled1d_supported(bb);
        case PCOT_JACOBI2D_5PT: return tiled2d_supported(bb);
        default: return tiled3d_supported(bb, dtype == PCOT_F64 ? 8 : dtype == PCOT_F32 ? 4 : 2);
    }
}

// ---------------------------------------------------------------- plans ---
struct DevPlan {
    std::vector<QEntry> host;
    QEntry* dev = nullptr;
    int device = -1;
    int64_t cnt[4] = {1, 1, 1, 1};
    ~DevPlan() {
        if (dev) (void)hipFree(dev);
    }
};

std::mutex g_mu;
std::map<std::vector<int64_t>, std::unique_ptr<DevPlan>> g_plans;

StencilGeom geom_of(const Prob& p) {
    int64_t tb[4] = {p.b[0], p.b[1], p.b[2], p.b[3]};
    if (p.kind == PCOT_FDTD2D) {
        // the embedded FDTD nest runs over all ny x nx cells: planned as a
        // stencil whose interior is that grid
        const int64_t n2[3] = {p.n[0] + 2, p.n[1] + 2, 1};
        return make_geom(p.d, n2, p.T, tb);
    }
    return make_geom(p.d, p.n, p.T, tb);
}

pcot_status get_plan(const Prob& p, DevPlan** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::vector<int64_t> key = {dev, p.d, p.n[0], p.n[1], p.n[2], p.T, p.b[0], p.b[1], p.b[2], p.b[3], p.sched,
                                p.kind == PCOT_FDTD2D};
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
        *out = it->second.get();
        return PCOT_OK;
    }
    StencilGeom g = geom_of(p);
    for (int i = 0; i <= p.d; ++i)
        if (g.cnt[i] >= 65535) return fail(PCOT_ERR_UNSUPPORTED, "tile grid too large along dim %d", i);
    std::vector<Leaf> leaves = enumerate_leaves(g, p.sched);
    auto P = std::make_unique<DevPlan>();
    P->device = dev;
    for (int i = 0; i < 4; ++i) P->cnt[i] = g.cnt[i];
    P->host.resize(leaves.size());
    for (size_t i = 0; i < leaves.size(); ++i)
        for (int j = 0; j < 4; ++j) P->host[i].k[j] = (uint16_t)leaves[i].k[j];
    if (!leaves.empty()) {
        HIP_TRY(hipMalloc(&P->dev, sizeof(QEntry) * leaves.size()));
        HIP_TRY(hipMemcpy(P->dev, P->host.data(), sizeof(QEntry) * leaves.size(), hipMemcpyHostToDevice));
    }
    *out = P.get();
    g_plans.emplace(key, std::move(P));
    return PCOT_OK;
}

// Trapezoid plans: built once per geometry on the host, uploaded per device.
struct TrapPlan {
    TrapPlanHost host;
    std::map<int, std::pair<TrapTile*, int*>> dev;
    ~TrapPlan() {
        for (auto& kv : dev) {
            if (kv.second.first) (void)hipFree(kv.second.first);
            if (kv.second.second) (void)hipFree(kv.second.second);
        }
    }
};
std::map<std::vector<int64_t>, std::unique_ptr<TrapPlan>> g_trap_plans;

TrapPlan* trap_plan_host(const Prob& p) {  // caller holds g_mu
    std::vector<int64_t> key = {p.n[0], p.n[1], p.T, p.b[0], p.b[1], p.b[2], p.sched};
    auto it = g_trap_plans.find(key);
    if (it != g_trap_plans.end()) return it->second.get();
    auto P = std::make_unique<TrapPlan>();
    const int F[2] = {p.b[1], p.b[2]};
    P->host = build_trap_plan((int)p.n[0], (int)p.n[1], (int)p.T, p.b[0], F, p.sched == PCOT_DIAMOND);
    TrapPlan* r = P.get();
    g_trap_plans.emplace(key, std::move(P));
    return r;
}

size_t trap_tile_count(const Prob& p) {
    std::lock_guard<std::mutex> lk(g_mu);
    return trap_plan_host(p)->host.tiles.size();
}

pcot_status get_trap_plan(const Prob& p, TrapPlan** out, TrapTile** dt, int** ds) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    TrapPlan* P = trap_plan_host(p);
    auto it = P->dev.find(dev);
    if (it == P->dev.end()) {
        TrapTile* t = nullptr;
        int* s = nullptr;
        const size_t nt = P->host.tiles.size(), ns = P->host.succ.size();
        if (nt) {
            HIP_TRY(hipMalloc(&t, sizeof(TrapTile) * nt));
            HIP_TRY(hipMemcpy(t, P->host.tiles.data(), sizeof(TrapTile) * nt, hipMemcpyHostToDevice));
        }
        if (ns) {
            HIP_TRY(hipMalloc(&s, sizeof(int) * ns));
            HIP_TRY(hipMemcpy(s, P->host.succ.data(), sizeof(int) * ns, hipMemcpyHostToDevice));
        }
        it = P->dev.emplace(dev, std::make_pair(t, s)).first;
    }
    *out = P;
    *dt = it->second.first;
    *ds = it->second.second;
    return PCOT_OK;
}

// ------------------------------------------------------------ workspace ---
struct WsLayout {
    size_t hdr = 0, probs = 0, counters = 0, field = 0, aux = 0, total = 0;
    size_t ncounters = 0;
};

WsLayout ws_layout(const Prob& p) {
    WsLayout L;
    L.hdr = 0;
    size_t off = align_up(HDR_WORDS * sizeof(unsigned));
    L.probs = off;
    off += align_up(sizeof(TiledProblem));
    if (is_trap(p.sched)) {
        const size_t nc = std::max<size_t>(1, trap_tile_count(p));
        L.ncounters = nc;
        L.counters = off;
        off += align_up(nc * sizeof(unsigned));
    } else if (p.sched != PCOT_NAIVE) {
        StencilGeom g = geom_of(p);
        size_t nc = 1;
        for (int i = 0; i <= p.d; ++i) nc *= (size_t)g.cnt[i];
        L.ncounters = nc;
        L.counters = off;
        off += align_up(nc * sizeof(unsigned));
    }
    L.field = off;
    if (!is_front(p.kind)) off += align_up((size_t)p.elems * elem_bytes(p.dtype));  // in-place kinds need none
    if (p.kind == PCOT_MOTIV1D) {  // Y[0..T], Z[0..T]
        L.aux = off;
        off += align_up(2 * (size_t)(p.T + 1) * sizeof(double));
    }
    L.total = off;
    return L;
}

TiledProblem make_tiled(const Prob& p, const DevPlan* plan, const void* in, void* out, void* ws_field,
                        unsigned* counters) {
    TiledProblem P;
    memset(&P, 0, sizeof P);
    P.in = in;
    // u_T lands in buf[T mod 2] = out
    if (p.T & 1) { P.buf1 = out; P.buf0 = ws_field; }
    else { P.buf0 = out; P.buf1 = ws_field; }
    for (int i = 0; i < 3; ++i) P.n[i] = (int)p.n[i];
    P.T = (int)p.T;
    for (int i = 0; i < 4; ++i) {
        P.b[i] = p.b[i];
        P.cnt[i] = (int)plan->cnt[i];
    }
    P.counters = counters;
    return P;
}

hipError_t launch_tiled_kind(int kind, int dtype, const int* b, const TiledLaunch& L, int grid_cap, hipStream_t s) {
    switch (kind) {
        case PCOT_JACOBI1D_3PT: return launch_tiled1d(dtype, b, L, grid_cap, s);
        case PCOT_JACOBI2D_5PT: return launch_tiled2d(dtype, b, L, grid_cap, s);
        default: return launch_tiled3d(dtype, b, L, grid_cap, s);
    }
}


// Optional timing of the dominant kernel of each run: an event pair recorded
// on the launch stream around the executor launch.
std::mutex g_tmu;
bool g_timing = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_events;

pcot_status timed_launch_begin(hipStream_t s, hipEvent_t* stop) {
    *stop = nullptr;
    if (!g_timing) return PCOT_OK;
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    HIP_TRY(hipEventRecord(a, s));
    std::lock_guard<std::mutex> lk(g_tmu);
    g_events.emplace_back(a, b);
    *stop = b;
    return PCOT_OK;
}

pcot_status timed_launch_end(hipStream_t s, hipEvent_t stop) {
    if (stop) HIP_TRY(hipEventRecord(stop, s));
    return PCOT_OK;
}

// --------------------------------------------------------------- DP plans ---
// Phases of (I, J) tiles over the upper triangle of nT x nT tiles; every tile's
// operands lie in tiles of earlier phases or in the tile itself.
//   wavefront: phase d = tile diagonal J - I = d;
//   recursive: a triangle splits into its two half triangles (concurrent,
//   merged phase by phase) followed by the square between them; a square
//   splits into bottom-left, then top-left and bottom-right (concurrent), then
//   top-right (the orthant recursion of Section 4.2 applied to the tile
//   triangle, with the parallel version's wavefront grouping).
using Phases = std::vector<std::vector<std::pair<int, int>>>;

void merge_into(Phases& dst, size_t at, const Phases& src) {
    if (dst.size() < at + src.size()) dst.resize(at + src.size());
    for (size_t k = 0; k < src.size(); ++k)
        dst[at + k].insert(dst[at + k].end(), src[k].begin(), src[k].end());
}

Phases dp_square(int i0, int j0, int n) {  // rows [i0, i0+n), cols [j0, j0+n)
    if (n == 1) return Phases{{{i0, j0}}};
    const int h = n / 2, r = n - h;
    // bottom-left: rows [i0+h, i0+n), cols [j0, j0+h)
    Phases out;
    Phases bl = dp_square(i0 + h, j0, std::min(h, r));
    (void)r;
    merge_into(out, 0, bl);
    Phases mid;
    merge_into(mid, 0, dp_square(i0, j0, h));
    merge_into(mid, 0, dp_square(i0 + h, j0 + h, h));
    merge_into(out, out.size(), mid);
    merge_into(out, out.size(), dp_square(i0, j0 + h, h));
    return out;
}

Phases dp_triangle(int i0, int n) {  // tiles (I, J), i0 <= I <= J < i0+n
    if (n == 1) return Phases{{{i0, i0}}};
    const int h = n / 2;
    Phases out;
    merge_into(out, 0, dp_triangle(i0, h));
    merge_into(out, 0, dp_triangle(i0 + h, h));
    merge_into(out, out.size(), dp_square(i0, i0 + h, h));
    return out;
}

// Per phase q, two launches: the external items of phase-q tiles whose
// operands include a tile of phase q-1 (`late`), then the finishing pass of
// phase q together with the external items of phase-(q+1) tiles whose
// operands were all finished by phase q-1 (`early`), which so run beside a
// finishing pass instead of after it.
struct DPPlan {
    int nT = 0, b = 0, kc = 0;
    std::vector<int> tile_off, late_off, early_off;  // per phase, into the arrays below
    std::vector<int2> tiles;
    std::vector<int4> late, early;
    int2* dtiles = nullptr;
    int4* dlate = nullptr;
    int4* dearly = nullptr;
    ~DPPlan() {
        if (dtiles) (void)hipFree(dtiles);
        if (dlate) (void)hipFree(dlate);
        if (dearly) (void)hipFree(dearly);
    }
};
std::map<std::vector<int64_t>, std::unique_ptr<DPPlan>> g_dp_plans;

pcot_status get_dp_plan(int nT, int b, int kc, int sched, DPPlan** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::vector<int64_t> key = {dev, nT, b, kc, sched};
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_dp_plans.find(key);
    if (it != g_dp_plans.end()) { *out = it->second.get(); return PCOT_OK; }
    Phases ph;
    if (sched == PCOT_SLT_WAVE) {
        ph.resize(nT);
        for (int d = 0; d < nT; ++d)
            for (int I = 0; I + d < nT; ++I) ph[d].push_back({I, I + d});
    } else {
        int p2 = 1;
        while (p2 < nT) p2 *= 2;
        // recursion over the padded power-of-two triangle, tiles past nT dropped
        Phases full = dp_triangle(0, p2);
        for (auto& q : full) {
            std::vector<std::pair<int, int>> keep;
            for (auto& t : q)
                if (t.second < nT) keep.push_back(t);
            if (!keep.empty()) ph.push_back(keep);
        }
    }
    auto P = std::make_unique<DPPlan>();
    P->nT = nT; P->b = b; P->kc = kc;
    const int nq = (int)ph.size();
    std::vector<int> phase_of((size_t)nT * nT, 0);
    for (int q = 0; q < nq; ++q)
        for (auto& t : ph[q]) phase_of[(size_t)t.first * nT + t.second] = q;
    std::vector<std::vector<int4>> late(nq), early(nq);
    for (int q = 0; q < nq; ++q)
        for (auto& t : ph[q]) {
            const int I = t.first, J = t.second;
            if (J == I) continue;
            const int k0 = (I + 1) * b - 1, k1 = J * b;  // external [k0, k1)
            for (int k = k0; k < k1; k += kc) {
                const int ke = std::min(k + kc, k1);
                // operands C[i][k'] in tiles (I, k'/b) and C[k'+1][j] in tiles ((k'+1)/b, J)
                int ready = 0;
                for (int K = k / b; K <= (ke - 1) / b; ++K) ready = std::max(ready, phase_of[(size_t)I * nT + K]);
                for (int K = (k + 1) / b; K <= ke / b; ++K) ready = std::max(ready, phase_of[(size_t)K * nT + J]);
                const int4 item = int4{(I << 16) | J, k, ke, 0};
                if (ready <= q - 2) early[q - 1].push_back(item);
                else late[q].push_back(item);
            }
        }
    for (int q = 0; q < nq; ++q) {
        P->tile_off.push_back((int)P->tiles.size());
        P->late_off.push_back((int)P->late.size());
        P->early_off.push_back((int)P->early.size());
        for (auto& t : ph[q]) P->tiles.push_back(int2{t.first, t.second});
        P->late.insert(P->late.end(), late[q].begin(), late[q].end());
        P->early.insert(P->early.end(), early[q].begin(), early[q].end());
    }
    P->tile_off.push_back((int)P->tiles.size());
    P->late_off.push_back((int)P->late.size());
    P->early_off.push_back((int)P->early.size());
    HIP_TRY(hipMalloc(&P->dtiles, sizeof(int2) * std::max<size_t>(1, P->tiles.size())));
    HIP_TRY(hipMemcpy(P->dtiles, P->tiles.data(), sizeof(int2) * P->tiles.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMalloc(&P->dlate, sizeof(int4) * std::max<size_t>(1, P->late.size())));
    if (!P->late.empty())
        HIP_TRY(hipMemcpy(P->dlate, P->late.data(), sizeof(int4) * P->late.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMalloc(&P->dearly, sizeof(int4) * std::max<size_t>(1, P->early.size())));
    if (!P->early.empty())
        HIP_TRY(hipMemcpy(P->dearly, P->early.data(), sizeof(int4) * P->early.size(), hipMemcpyHostToDevice));
    *out = P.get();
    g_dp_plans.emplace(key, std::move(P));
    return PCOT_OK;
}

struct DPArgs {
    int64_t N = 0, Np = 0;
    int b = 64, kc = 256;
    bool wide = false;
    size_t hdr = 0, pp = 0, cw = 0, total = 0;
};

pcot_status dp_validate(int64_t N, int64_t pmax, const pcot_tile* tile, int32_t schedule, DPArgs& A) {
    if (N < 1 || N > 65536) return fail(PCOT_ERR_INVALID, "N=%lld out of range 1..65536", (long long)N);
    if (schedule != PCOT_SLT_WAVE && schedule != PCOT_COT_PAR)
        return fail(PCOT_ERR_INVALID, "DP schedules: PCOT_SLT_WAVE or PCOT_COT_PAR");
    A.N = N;
    if (tile) {
        A.b = tile->s[0];
        A.kc = tile->s[2] > 0 ? tile->s[2] : 256;
        if (tile->s[1] != tile->s[0]) return fail(PCOT_ERR_INVALID, "DP tiles are square: s[0] == s[1]");
    }
    if (!dp_block_supported(A.b)) return fail(PCOT_ERR_UNSUPPORTED, "DP block size %d (supported: 16, 32, 64)", A.b);
    if (A.kc < 16 || A.kc % 16) return fail(PCOT_ERR_INVALID, "DP k-chunk %d: multiple of 16 required", A.kc);
    A.Np = (N + A.b - 1) / A.b * A.b;
    {
        // external items (one per tile pair and k-chunk of the off-diagonal
        // k range) are indexed with int offsets in the plan: bound their count
        const int64_t nT = A.Np / A.b;
        int64_t items = 0;
        for (int64_t d = 1; d < nT; ++d)
            items += (nT - d) * (((d - 1) * A.b + 1 + A.kc - 1) / A.kc);
        if (items > (int64_t)INT32_MAX)
            return fail(PCOT_ERR_UNSUPPORTED, "DP plan of %lld k-chunk items exceeds 2^31-1 (use a larger k-chunk or block)",
                        (long long)items);
    }
    // exactness: every candidate is at most (N-1) * pmax^3
    const long double bound = (long double)(N > 1 ? N - 1 : 1) * (long double)pmax * pmax * pmax;
    if (pmax < 1) return fail(PCOT_ERR_INVALID, "pmax=%lld < 1", (long long)pmax);
    if (bound >= 4611686018427387904.0L) return fail(PCOT_ERR_OVERFLOW, "(N-1)*pmax^3 >= 2^62");
    A.wide = bound >= 4294967296.0L;
    const size_t es = A.wide ? 8 : 4;
    A.hdr = 0;
    A.pp = align_up(HDR_WORDS * sizeof(unsigned));
    A.cw = A.pp + align_up(sizeof(int64_t) * (A.Np + 1));
    A.total = A.cw + align_up(es * (size_t)A.Np * A.Np);
    return PCOT_OK;
}

// ---------------------------------------------------------------- batches ---
// A batch shares kind, dtype and schedule; the persistent launch needs one
// kernel instance, so the tiles share the launch shape (b_x, and b_y for
// Heat-3D, whose block is b_y waves) while b_t and the other sizes may
// differ per instance.
struct BatchPlan {
    std::vector<QEntry> host;
    std::vector<uint16_t> hprob;
    std::vector<std::array<int64_t, 4>> cnt;
    QEntry* dev = nullptr;
    uint16_t* devp = nullptr;
    ~BatchPlan() {
        if (dev) (void)hipFree(dev);
        if (devp) (void)hipFree(devp);
    }
};
std::map<std::vector<int64_t>, std::unique_ptr<BatchPlan>> g_bplans;

struct Batch {
    std::vector<Prob> p;
    int lb[4] = {1, 1, 1, 1};  // launch shape
};

pcot_status batch_validate(int32_t kind, int32_t dtype, int32_t n, const int64_t* dims, const int64_t* T,
                           const pcot_tile* tiles, int32_t schedule, Batch& B) {
    if (n < 1 || n > 65535) return fail(PCOT_ERR_INVALID, "batch of %d instances (need 1 .. 65535)", n);
    if (!dims || !T || !tiles) return fail(PCOT_ERR_INVALID, "dims/T/tiles is NULL");
    if (schedule == PCOT_NAIVE) return fail(PCOT_ERR_UNSUPPORTED, "batched runs need a tiled schedule");
    if (is_trap(schedule)) return fail(PCOT_ERR_UNSUPPORTED, "batched runs take the box-tile schedules (1..4)");
    if (is_front(kind) || kind == PCOT_MOTIV1D)
        return fail(PCOT_ERR_UNSUPPORTED, "batched runs take the Jacobi and Heat-3D kinds");
    B.p.resize(n);
    for (int i = 0; i < n; ++i) {
        pcot_status st = validate(kind, dtype, dims + 3 * (size_t)i, T[i], tiles + i, schedule, B.p[i]);
        if (st != PCOT_OK) return fail(st, "instance %d: %s", i, g_err.c_str());
        if (!tile_ok(kind, dtype, B.p[i].b)) return fail(PCOT_ERR_UNSUPPORTED, "instance %d: tile not runnable", i);
    }
    const Prob& p0 = B.p[0];
    const int d = p0.d;
    for (int j = 0; j < 4; ++j) B.lb[j] = p0.b[j];
    for (int i = 1; i < n; ++i) {
        const Prob& q = B.p[i];
        if (q.b[d] != p0.b[d]) return fail(PCOT_ERR_UNSUPPORTED, "instance %d: b_x differs within the batch", i);
        if (d == 3 && q.b[2] != p0.b[2]) return fail(PCOT_ERR_UNSUPPORTED, "instance %d: b_y differs within the batch", i);
        for (int j = 0; j < d; ++j) B.lb[j] = std::max(B.lb[j], q.b[j]);
    }
    if (!tile_ok(kind, dtype, B.lb)) return fail(PCOT_ERR_UNSUPPORTED, "no executor instance covers the batch's largest tile");
    return PCOT_OK;
}

struct BatchLayout {
    size_t hdr = 0, probs = 0, counters = 0, ncounters = 0, total = 0;
    std::vector<size_t> cnt_off, field_off;
};

BatchLayout batch_layout(const Batch& B) {
    BatchLayout L;
    const size_t n = B.p.size();
    size_t off = align_up(HDR_WORDS * sizeof(unsigned));
    L.probs = off;
    off += align_up(n * sizeof(TiledProblem));
    L.counters = off;
    size_t c = 0;
    for (const Prob& p : B.p) {
        StencilGeom g = geom_of(p);
        size_t nc = 1;
        for (int i = 0; i <= p.d; ++i) nc *= (size_t)g.cnt[i];
        L.cnt_off.push_back(c);
        c += (nc + 63) / 64 * 64;
    }
    L.ncounters = c;
    off += align_up(c * sizeof(unsigned));
    for (const Prob& p : B.p) {
        L.field_off.push_back(off);
        off += align_up((size_t)p.elems * elem_bytes(p.dtype));
    }
    L.total = off;
    return L;
}

// Leaves of all instances merged by fractional progress: leaf j of an
// instance with m leaves gets key (j + 1/2) / m, so every instance advances
// through its own order at the same relative pace and all finish near the end
// of the queue; ties go to the instance with more updates.  Each instance's
// own order is kept, so the merged queue stays topological.
pcot_status get_batch_plan(const Batch& B, int sched, BatchPlan** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::vector<int64_t> key = {dev, B.p[0].d, sched, (int64_t)B.p.size()};
    for (const Prob& p : B.p) {
        key.insert(key.end(), {p.n[0], p.n[1], p.n[2], p.T, p.b[0], p.b[1], p.b[2], p.b[3]});
    }
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_bplans.find(key);
    if (it != g_bplans.end()) {
        *out = it->second.get();
        return PCOT_OK;
    }
    auto P = std::make_unique<BatchPlan>();
    struct Item {
        double key;
        int64_t weight;
        int inst;
        QEntry e;
    };
    std::vector<Item> items;
    for (size_t i = 0; i < B.p.size(); ++i) {
        const Prob& p = B.p[i];
        StencilGeom g = geom_of(p);
        for (int j = 0; j <= p.d; ++j)
            if (g.cnt[j] >= 65535) return fail(PCOT_ERR_UNSUPPORTED, "instance %zu: tile grid too large", i);
        P->cnt.push_back({g.cnt[0], g.cnt[1], g.cnt[2], g.cnt[3]});
        int64_t w = p.T;
        for (int j = 0; j < p.d; ++j) w *= p.n[j] - 2;
        std::vector<Leaf> leaves = enumerate_leaves(g, sched);
        const double m = (double)leaves.size();
        for (size_t j = 0; j < leaves.size(); ++j) {
            Item it2;
            it2.key = ((double)j + 0.5) / m;
            it2.weight = w;
            it2.inst = (int)i;
            for (int q = 0; q < 4; ++q) it2.e.k[q] = (uint16_t)leaves[j].k[q];
            items.push_back(it2);
        }
    }
    std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) {
        if (a.key != b.key) return a.key < b.key;
        if (a.weight != b.weight) return a.weight > b.weight;
        return a.inst < b.inst;
    });
    for (const Item& x : items) {
        P->host.push_back(x.e);
        P->hprob.push_back((uint16_t)x.inst);
    }
    if (!items.empty()) {
        HIP_TRY(hipMalloc(&P->dev, sizeof(QEntry) * items.size()));
        HIP_TRY(hipMemcpy(P->dev, P->host.data(), sizeof(QEntry) * items.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMalloc(&P->devp, sizeof(uint16_t) * items.size()));
        HIP_TRY(hipMemcpy(P->devp, P->hprob.data(), sizeof(uint16_t) * items.size(), hipMemcpyHostToDevice));
    }
    *out = P.get();
    g_bplans.emplace(key, std::move(P));
    return PCOT_OK;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + nb && y < x + na;
}

// Binary64 error norms: one scratch buffer per device, made on first use.
std::mutex g_nmu;
std::map<int, double*> g_norm_scratch;

}  // namespace

extern "C" {

const char* pcot_last_error(void) { return g_err.c_str(); }
const char* pcot_version(void) { return "pcot-mi355x 0.1 (gfx950)"; }

size_t pcot_stencil_workspace(int32_t kind, int32_t dtype, const int64_t* dims, int64_t T, const pcot_tile* tile,
                              int32_t schedule) {
    PCOT_TRY
    Prob p;
    if (validate(kind, dtype, dims, T, tile, schedule, p) != PCOT_OK) return 0;
    return ws_layout(p).total;
    PCOT_CATCH(0)
}

pcot_status pcot_stencil_tile_supported(int32_t kind, int32_t dtype, const pcot_tile* tile) {
    PCOT_TRY
    const int d = kind_dims(kind);
    if (!d) return fail(PCOT_ERR_INVALID, "unknown kind %d", kind);
    if (dtype < PCOT_F64 || dtype > PCOT_BF16) return fail(PCOT_ERR_INVALID, "unknown dtype %d", dtype);
    if (!tile || tile->t < 1) return fail(PCOT_ERR_INVALID, "bad tile");
    int b[4] = {tile->t, 1, 1, 1};
    for (int i = 0; i < d; ++i) {
        if (tile->s[i] < 2) return fail(PCOT_ERR_INVALID, "tile.s[%d] < 2", i);
        b[i + 1] = tile->s[i];
    }
    if (!tile_ok(kind, dtype, b)) return fail(PCOT_ERR_UNSUPPORTED, "tile (%d; %d,%d,%d) not runnable for kind %d dtype %d", b[0], b[1], b[2], b[3], kind, dtype);
    return PCOT_OK;
    PCOT_CATCH(PCOT_ERR_HOST)
}

int64_t pcot_stencil_plan(int32_t kind, const int64_t* dims, int64_t T, const pcot_tile* tile, int32_t schedule,
                          int32_t* order, int64_t cap) {
    PCOT_TRY
    Prob p;
    if (schedule == PCOT_NAIVE) { fail(PCOT_ERR_INVALID, "naive schedule has no plan"); return -1; }
    if (is_trap(schedule)) { fail(PCOT_ERR_INVALID, "trapezoid plans: pcot_stencil_trap_plan"); return -1; }
    if (validate(kind, PCOT_F64, dims, T, tile, schedule, p) != PCOT_OK) return -1;
    StencilGeom g = geom_of(p);
    std::vector<Leaf> leaves = enumerate_leaves(g, schedule);
    if (order)
        for (int64_t i = 0; i < (int64_t)leaves.size() && i < cap; ++i)
            for (int j = 0; j < 4; ++j) order[4 * i + j] = leaves[i].k[j];
    return (int64_t)leaves.size();
    PCOT_CATCH(-1)
}

int64_t pcot_stencil_trap_plan(const int64_t* dims, int64_t T, const pcot_tile* tile, int32_t schedule,
                               int32_t* tiles, int64_t cap, int32_t* edges, int64_t edge_cap, int64_t* n_edges,
                               int64_t* traffic) {
    PCOT_TRY
    Prob p;
    if (!is_trap(schedule)) { fail(PCOT_ERR_INVALID, "schedule %d is not a trapezoid schedule", schedule); return -1; }
    if (validate(PCOT_JACOBI2D_5PT, PCOT_F64, dims, T, tile, schedule, p) != PCOT_OK) return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    const TrapPlanHost& H = trap_plan_host(p)->host;
    const int64_t nt = (int64_t)H.tiles.size();
    if (tiles)
        for (int64_t i = 0; i < nt && i < cap; ++i) {
            const TrapTile& t = H.tiles[i];
            const int32_t rec[12] = {t.lo[0], t.hi[0], t.slo[0], t.shi[0], t.fo[0], t.lo[1],
                                     t.hi[1], t.slo[1], t.shi[1], t.fo[1], t.t0, t.nt};
            memcpy(tiles + 12 * i, rec, sizeof rec);
        }
    int64_t ne = 0;
    for (int64_t i = 0; i < nt; ++i)
        for (int k = 0; k < H.tiles[i].nsucc; ++k, ++ne)
            if (edges && ne < edge_cap) {
                edges[2 * ne] = (int32_t)i;
                edges[2 * ne + 1] = H.succ[H.tiles[i].succ0 + k];
            }
    if (n_edges) *n_edges = ne;
    if (traffic) {
        traffic[0] = H.loads;
        traffic[1] = H.stores;
    }
    return nt;
    PCOT_CATCH(-1)
}

pcot_status pcot_stencil_run(int32_t kind, int32_t dtype, const int64_t* dims, int64_t T, const pcot_tile* tile,
                             int32_t schedule, const void* in, void* out, void* workspace, size_t ws_bytes,
                             void* stream) {
    PCOT_TRY
    Prob p;
    pcot_status st = validate(kind, dtype, dims, T, tile, schedule, p);
    if (st != PCOT_OK) return st;
    if (!in || !out) return fail(PCOT_ERR_INVALID, "in/out is NULL");
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = (size_t)p.elems * elem_bytes(dtype) * kind_fields(kind);
    {
        const char* a = (const char*)in;
        const char* b = (const char*)out;
        if (a < b + bytes && b < a + bytes) return fail(PCOT_ERR_INVALID, "in and out overlap");
    }
    if (schedule != PCOT_NAIVE && !tile_ok(kind, dtype, p.b, schedule))
        return fail(PCOT_ERR_UNSUPPORTED, "tile (%d; %d,%d,%d) not runnable for kind %d dtype %d", p.b[0], p.b[1],
                    p.b[2], p.b[3], kind, dtype);
    if (T == 0) {
        HIP_TRY(hipMemcpyAsync(out, in, bytes, hipMemcpyDeviceToDevice, s));
        return PCOT_OK;
    }
    const WsLayout W = ws_layout(p);
    if (!workspace || ws_bytes < W.total)
        return fail(PCOT_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, W.total);
    if (((uintptr_t)workspace) % ALIGN) return fail(PCOT_ERR_INVALID, "workspace not 256-byte aligned");
    char* ws = (char*)workspace;
    unsigned* hdr = (unsigned*)(ws + W.hdr);
    void* field = ws + W.field;
    {
        const char* a = (const char*)workspace;
        const char* b = (const char*)out;
        if (a < b + bytes && b < a + W.total) return fail(PCOT_ERR_INVALID, "out overlaps the workspace");
        const char* c = (const char*)in;
        if (a < c + bytes && c < a + W.total) return fail(PCOT_ERR_INVALID, "in overlaps the workspace");
    }
    if (is_front(kind)) {
        // in place on out: every field copied first
        HIP_TRY(hipMemcpyAsync(out, in, bytes, hipMemcpyDeviceToDevice, s));
        const size_t fe = (size_t)p.elems;
        double* f0 = (double*)out;
        if (schedule == PCOT_NAIVE) {  // FDTD-2D only (validated)
            for (int64_t t = 0; t < T; ++t)
                HIP_TRY(launch_fdtd2d_step(f0, f0 + fe, f0 + 2 * fe, (int)p.n[0], (int)p.n[1], s));
            return PCOT_OK;
        }
        DevPlan* plan = nullptr;
        st = get_plan(p, &plan);
        if (st != PCOT_OK) return st;
        unsigned* counters = (unsigned*)(ws + W.counters);
        HIP_TRY(launch_fill_u32(hdr, HDR_WORDS, 0u, s));
        HIP_TRY(launch_fill_u32(counters, W.ncounters, 0u, s));
        if (plan->host.empty()) return PCOT_OK;
        TiledProblem P = make_tiled(p, plan, f0, f0, f0, counters);
        if (kind == PCOT_FDTD2D) {
            // ex, ey, hz; the planner's extents include the embedding's frame
            P.buf0 = f0;
            P.buf1 = f0 + fe;
            P.in = f0 + 2 * fe;
            P.n[0] = (int)p.n[0] + 2;
            P.n[1] = (int)p.n[1] + 2;
        }
        TiledProblem* probs = (TiledProblem*)(ws + W.probs);
        HIP_TRY(launch_put_problem(probs, P, s));
        TiledLaunch L;
        memset(&L, 0, sizeof L);
        L.probs = probs;
        L.queue = plan->dev;
        L.nq = (int)plan->host.size();
        L.hdr = hdr;
        L.limit_ticks = watchdog_ticks();
        hipEvent_t stop;
        st = timed_launch_begin(s, &stop);
        if (st != PCOT_OK) return st;
        HIP_TRY(launch_front2d(kind, p.b, L, s));
        return timed_launch_end(s, stop);
    }
    if (kind == PCOT_MOTIV1D) {
        double* Y = (double*)(ws + W.aux);
        double* Z = Y + (T + 1);
        const int N = (int)p.n[0];
        HIP_TRY(launch_motiv_boundary((const double*)in, Y, Z, (double*)out, N, (int)T, s));
        void* buf[2];
        buf[T & 1] = out;
        buf[(T + 1) & 1] = field;
        if (schedule == PCOT_NAIVE) {
            for (int64_t t = 0; t < T; ++t)
                HIP_TRY(launch_motiv_step((const double*)(t == 0 ? in : buf[t & 1]), (double*)buf[(t + 1) & 1], Y,
                                          Z, N, (int)t, s));
            return PCOT_OK;
        }
        DevPlan* plan = nullptr;
        st = get_plan(p, &plan);
        if (st != PCOT_OK) return st;
        unsigned* counters = (unsigned*)(ws + W.counters);
        HIP_TRY(launch_fill_u32(hdr, HDR_WORDS, 0u, s));
        HIP_TRY(launch_fill_u32(counters, W.ncounters, 0u, s));
        if (plan->host.empty()) return PCOT_OK;
        TiledProblem* probs = (TiledProblem*)(ws + W.probs);
        HIP_TRY(launch_put_problem(probs, make_tiled(p, plan, in, out, field, counters), s));
        TiledLaunch L;
        memset(&L, 0, sizeof L);
        L.probs = probs;
        L.queue = plan->dev;
        L.nq = (int)plan->host.size();
        L.hdr = hdr;
        L.limit_ticks = watchdog_ticks();
        hipEvent_t stop;
        st = timed_launch_begin(s, &stop);
        if (st != PCOT_OK) return st;
        HIP_TRY(launch_motiv_tiles(p.b, L, Y, Z, s));
        return timed_launch_end(s, stop);
    }
    // buffers: buf[T mod 2] = out, the other one in the workspace; both get in's boundary
    HIP_TRY(launch_copy_boundary(dtype, in, out, field, p.d, p.n, s));
    if (schedule == PCOT_NAIVE && kind == PCOT_JACOBI1D_3PT && resident1d_fits(dtype, p.n[0])) {
        // the whole field stays in one CU's LDS for all T steps: one launch
        HIP_TRY(launch_fill_u32(hdr, HDR_WORDS, 0u, s));
        HIP_TRY(launch_resident1d(dtype, in, out, (int)p.n[0], (int)T, s));
        return PCOT_OK;
    }
    if (schedule == PCOT_NAIVE) {
        HIP_TRY(launch_fill_u32(hdr, HDR_WORDS, 0u, s));
        void* buf[2];
        buf[T & 1] = out;
        buf[(T + 1) & 1] = field;
        for (int64_t t = 0; t < T; ++t) {
            const void* src = t == 0 ? in : buf[t & 1];
            HIP_TRY(launch_step(kind, dtype, src, buf[(t + 1) & 1], p.n, s));
        }
        return PCOT_OK;
    }
    if (is_trap(schedule)) {
        TrapPlan* tp = nullptr;
        TrapTile* dt = nullptr;
        int* ds = nullptr;
        st = get_trap_plan(p, &tp, &dt, &ds);
        if (st != PCOT_OK) return st;
        unsigned* counters = (unsigned*)(ws + W.counters);
        HIP_TRY(launch_fill_u32(hdr, HDR_WORDS, 0u, s));
        HIP_TRY(launch_fill_u32(counters, W.ncounters, 0u, s));
        if (tp->host.tiles.empty()) return PCOT_OK;
        TrapLaunch L;
        memset(&L, 0, sizeof L);
        L.tiles = dt;
        L.succ = ds;
        L.counters = counters;
        L.hdr = hdr;
        L.in = in;
        // u_T lands in buf[T mod 2] = out
        L.buf0 = (T & 1) ? field : out;
        L.buf1 = (T & 1) ? out : field;
        L.ntiles = (int)tp->host.tiles.size();
        L.ny = (int)p.n[0];
        L.nx = (int)p.n[1];
        L.limit_ticks = watchdog_ticks();
        hipEvent_t stop;
        st = timed_launch_begin(s, &stop);
        if (st != PCOT_OK) return st;
        HIP_TRY(launch_trap2d(dtype, p.b[0], p.b[1], p.b[2], L, s));
        return timed_launch_end(s, stop);
    }
    DevPlan* plan = nullptr;
    st = get_plan(p, &plan);
    if (st != PCOT_OK) return st;
    unsigned* counters = (unsigned*)(ws + W.counters);
    HIP_TRY(launch_fill_u32(hdr, HDR_WORDS, 0u, s));
    HIP_TRY(launch_fill_u32(counters, W.ncounters, 0u, s));
    if (plan->host.empty()) return PCOT_OK;
    TiledProblem* probs = (TiledProblem*)(ws + W.probs);
    HIP_TRY(launch_put_problem(probs, make_tiled(p, plan, in, out, field, counters), s));
    TiledLaunch L;
    memset(&L, 0, sizeof L);
    L.probs = probs;
    L.queue = plan->dev;
    L.qprob = nullptr;
    L.nq = (int)plan->host.size();
    L.hdr = hdr;
    L.limit_ticks = watchdog_ticks();
    hipEvent_t stop;
    st = timed_launch_begin(s, &stop);
    if (st != PCOT_OK) return st;
    HIP_TRY(launch_tiled_kind(kind, dtype, p.b, L, 0, s));
    return timed_launch_end(s, stop);
    PCOT_CATCH(PCOT_ERR_HOST)
}

size_t pcot_stencil_workspace_batched(int32_t kind, int32_t dtype, int32_t n, const int64_t* dims,
                                      const int64_t* T, const pcot_tile* tiles, int32_t schedule) {
    PCOT_TRY
    Batch B;
    if (batch_validate(kind, dtype, n, dims, T, tiles, schedule, B) != PCOT_OK) return 0;
    return batch_layout(B).total;
    PCOT_CATCH(0)
}

pcot_status pcot_stencil_run_batched(int32_t kind, int32_t dtype, int32_t n, const int64_t* dims,
                                     const int64_t* T, const pcot_tile* tiles, int32_t schedule,
                                     const void* const* in, void* const* out, void* workspace, size_t ws_bytes,
                                     void* stream) {
    PCOT_TRY
    Batch B;
    pcot_status st = batch_validate(kind, dtype, n, dims, T, tiles, schedule, B);
    if (st != PCOT_OK) return st;
    if (!in || !out) return fail(PCOT_ERR_INVALID, "in/out is NULL");
    const BatchLayout W = batch_layout(B);
    if (!workspace || ws_bytes < W.total)
        return fail(PCOT_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, W.total);
    if (((uintptr_t)workspace) % ALIGN) return fail(PCOT_ERR_INVALID, "workspace not 256-byte aligned");
    for (int i = 0; i < n; ++i) {
        const size_t bytes = (size_t)B.p[i].elems * elem_bytes(dtype);
        if (!in[i] || !out[i]) return fail(PCOT_ERR_INVALID, "instance %d: in/out is NULL", i);
        if (overlaps(in[i], bytes, out[i], bytes)) return fail(PCOT_ERR_INVALID, "instance %d: in and out overlap", i);
        if (overlaps(out[i], bytes, workspace, W.total) || overlaps(in[i], bytes, workspace, W.total))
            return fail(PCOT_ERR_INVALID, "instance %d: in/out overlaps the workspace", i);
    }
    BatchPlan* plan = nullptr;
    st = get_batch_plan(B, schedule, &plan);
    if (st != PCOT_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)workspace;
    unsigned* hdr = (unsigned*)(ws + W.hdr);
    unsigned* counters = (unsigned*)(ws + W.counters);
    TiledProblem* probs = (TiledProblem*)(ws + W.probs);
    std::vector<TiledProblem> hp(n);
    for (int i = 0; i < n; ++i) {
        const Prob& p = B.p[i];
        TiledProblem& P = hp[i];
        memset(&P, 0, sizeof P);
        P.in = in[i];
        void* field = ws + W.field_off[i];
        if (p.T & 1) { P.buf1 = out[i]; P.buf0 = field; }
        else { P.buf0 = out[i]; P.buf1 = field; }
        for (int j = 0; j < 3; ++j) P.n[j] = (int)p.n[j];
        P.T = (int)p.T;
        for (int j = 0; j < 4; ++j) {
            P.b[j] = p.b[j];
            P.cnt[j] = (int)plan->cnt[i][j];
        }
        P.counters = counters + W.cnt_off[i];
    }
    HIP_TRY(launch_fill_u32(hdr, HDR_WORDS, 0u, s));
    HIP_TRY(launch_fill_u32(counters, W.ncounters, 0u, s));
    HIP_TRY(launch_put_problems(probs, hp.data(), n, s));
    HIP_TRY(launch_copy_boundary_batched(dtype, probs, n, B.p[0].d, s));
    for (int i = 0; i < n; ++i)
        if (B.p[i].T == 0)
            HIP_TRY(hipMemcpyAsync(out[i], in[i], (size_t)B.p[i].elems * elem_bytes(dtype), hipMemcpyDeviceToDevice, s));
    if (plan->host.empty()) return PCOT_OK;
    TiledLaunch L;
    memset(&L, 0, sizeof L);
    L.probs = probs;
    L.queue = plan->dev;
    L.qprob = plan->devp;
    L.nq = (int)plan->host.size();
    L.hdr = hdr;
    L.limit_ticks = watchdog_ticks();
    hipEvent_t stop;
    st = timed_launch_begin(s, &stop);
    if (st != PCOT_OK) return st;
    HIP_TRY(launch_tiled_kind(kind, dtype, B.lb, L, 0, s));
    return timed_launch_end(s, stop);
    PCOT_CATCH(PCOT_ERR_HOST)
}

pcot_status pcot_error_norms(int32_t dtype, int32_t d, const int64_t* dims, const void* x, const double* r,
                             double* out, void* stream) {
    PCOT_TRY
    if (dtype < PCOT_F64 || dtype > PCOT_BF16) return fail(PCOT_ERR_INVALID, "unknown dtype %d", dtype);
    if (d < 1 || d > 3) return fail(PCOT_ERR_INVALID, "d=%d (need 1..3)", d);
    if (!dims || !x || !r || !out) return fail(PCOT_ERR_INVALID, "NULL argument");
    int64_t n[3] = {1, 1, 1};
    for (int i = 0; i < d; ++i) {
        if (dims[i] < 3 || dims[i] > (1LL << 30)) return fail(PCOT_ERR_INVALID, "dims[%d]=%lld", i, (long long)dims[i]);
        n[i] = dims[i];
    }
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_nmu);
    double*& scratch = g_norm_scratch[dev];
    if (!scratch) HIP_TRY(hipMalloc(&scratch, norms_scratch_bytes()));
    HIP_TRY(launch_norms(dtype, d, n, x, r, scratch, s));
    const size_t res = norms_scratch_bytes() / sizeof(double) - 4;
    HIP_TRY(hipMemcpyAsync(out, scratch + res, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return PCOT_OK;
    PCOT_CATCH(PCOT_ERR_HOST)
}

pcot_status pcot_error_norms_static(int32_t dtype, int32_t d, const int64_t* dims, const void* x,
                                    const double* r, double* out, void* stream) {
    PCOT_TRY
    if (dtype < PCOT_F64 || dtype > PCOT_BF16) return fail(PCOT_ERR_INVALID, "unknown dtype %d", dtype);
    if (d < 1 || d > 3) return fail(PCOT_ERR_INVALID, "d=%d (need 1..3)", d);
    if (!dims || !x || !r || !out) return fail(PCOT_ERR_INVALID, "NULL argument");
    int64_t n[3] = {1, 1, 1};
    for (int i = 0; i < d; ++i) {
        if (dims[i] < 3 || dims[i] > (1LL << 30)) return fail(PCOT_ERR_INVALID, "dims[%d]=%lld", i, (long long)dims[i]);
        n[i] = dims[i];
    }
    const double total = (double)(n[0] - 2) * (double)(d >= 2 ? n[1] - 2 : 1) * (double)(d >= 3 ? n[2] - 2 : 1);
    if (total > (double)PCOT_NORMS_STATIC_MAX_POINTS)
        return fail(PCOT_ERR_UNSUPPORTED, "%.0f interior points exceed the allocation-free limit %lld", total,
                    (long long)PCOT_NORMS_STATIC_MAX_POINTS);
    double* scratch = nullptr;
    HIP_TRY(norms_static_scratch(&scratch));
    HIP_TRY(launch_norms_to(dtype, d, n, x, r, scratch, out, (hipStream_t)stream));
    return PCOT_OK;
    PCOT_CATCH(PCOT_ERR_HOST)
}

size_t pcot_dp_workspace(int64_t N, const pcot_tile* tile, int32_t schedule) {
    PCOT_TRY
    DPArgs A;
    // the 64-bit working matrix is the larger case; size for it
    if (dp_validate(N, 1, tile, schedule, A) != PCOT_OK) return 0;
    return A.cw + align_up(8 * (size_t)A.Np * A.Np);
    PCOT_CATCH(0)
}

pcot_status pcot_dp_run(const int64_t* p, int64_t N, int64_t pmax, const pcot_tile* tile, int32_t schedule,
                        int64_t* C, void* workspace, size_t ws_bytes, void* stream) {
    PCOT_TRY
    DPArgs A;
    pcot_status st = dp_validate(N, pmax, tile, schedule, A);
    if (st != PCOT_OK) return st;
    if (!p || !C) return fail(PCOT_ERR_INVALID, "p/C is NULL");
    if (!workspace || ws_bytes < A.total) return fail(PCOT_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, A.total);
    if (((uintptr_t)workspace) % ALIGN) return fail(PCOT_ERR_INVALID, "workspace not 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)workspace;
    DPPlan* plan = nullptr;
    st = get_dp_plan((int)(A.Np / A.b), A.b, A.kc, schedule, &plan);
    if (st != PCOT_OK) return st;
    DPLaunch L;
    memset(&L, 0, sizeof L);
    L.p = (const long long*)(ws + A.pp);
    L.Cw = ws + A.cw;
    L.C = (long long*)C;
    L.N = (int)A.Np;
    L.Nout = (int)N;
    L.b = A.b;
    L.hdr = (unsigned*)(ws + A.hdr);
    L.pmax = pmax;
    HIP_TRY(launch_fill_u32(L.hdr, HDR_WORDS, 0u, s));
    HIP_TRY(launch_dp_pad((const long long*)p, (long long*)(ws + A.pp), (int)N, (int)A.Np, s));
    HIP_TRY(launch_dp_phase(A.wide, L, DP_INIT, s));
    hipEvent_t stop;
    st = timed_launch_begin(s, &stop);
    if (st != PCOT_OK) return st;
    for (size_t q = 0; q + 1 < plan->tile_off.size(); ++q) {
        L.tiles = plan->dtiles;
        L.ntiles = 0;
        L.items = plan->dlate + plan->late_off[q];
        L.nitems = plan->late_off[q + 1] - plan->late_off[q];
        HIP_TRY(launch_dp_phase(A.wide, L, DP_ITEMS, s));
        L.tiles = plan->dtiles + plan->tile_off[q];
        L.ntiles = plan->tile_off[q + 1] - plan->tile_off[q];
        L.items = plan->dearly + plan->early_off[q];
        L.nitems = plan->early_off[q + 1] - plan->early_off[q];
        HIP_TRY(launch_dp_phase(A.wide, L, DP_FINISH, s));
    }
    return timed_launch_end(s, stop);
    PCOT_CATCH(PCOT_ERR_HOST)
}

pcot_status pcot_dp_split(const int64_t* p, int64_t N, const int64_t* C, int64_t* split, void* stream) {
    PCOT_TRY
    if (N < 1 || N > 65535) return fail(PCOT_ERR_INVALID, "N=%lld (need 1 .. 65535)", (long long)N);
    if (!p || !C || !split) return fail(PCOT_ERR_INVALID, "p/C/split is NULL");
    HIP_TRY(launch_dp_split((const long long*)p, (const long long*)C, (long long*)split, (int)N,
                            (hipStream_t)stream));
    return PCOT_OK;
    PCOT_CATCH(PCOT_ERR_HOST)
}

pcot_status pcot_stream_status(void* workspace, void* stream) {
    PCOT_TRY
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    if (!workspace) return fail(PCOT_ERR_INVALID, "workspace is NULL");
    unsigned w = 0;
    HIP_TRY(hipMemcpy(&w, (unsigned*)workspace + HDR_ERROR, sizeof w, hipMemcpyDeviceToHost));
    if (w == DEVERR_TIMEOUT) return fail(PCOT_ERR_TIMEOUT, "device watchdog: a tile waited more than 4 s for its inputs");
    if (w == DEVERR_INPUT) return fail(PCOT_ERR_DEVICE, "device validation failed (input out of the stated range)");
    if (w != 0) return fail(PCOT_ERR_DEVICE, "device error word %u", w);
    return PCOT_OK;
    PCOT_CATCH(PCOT_ERR_HOST)
}

pcot_status pcot_kernel_timing(int32_t enable) {
    PCOT_TRY
    std::lock_guard<std::mutex> lk(g_tmu);
    for (auto& e : g_events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    g_events.clear();
    g_timing = enable != 0;
    return PCOT_OK;
    PCOT_CATCH(PCOT_ERR_HOST)
}

pcot_status pcot_kernel_timing_read(double* total_ms, int64_t* count) {
    PCOT_TRY
    std::lock_guard<std::mutex> lk(g_tmu);
    double tot = 0.0;
    for (auto& e : g_events) {
        HIP_TRY(hipEventSynchronize(e.second));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e.first, e.second));
        tot += ms;
    }
    if (total_ms) *total_ms = tot;
    if (count) *count = (int64_t)g_events.size();
    return PCOT_OK;
    PCOT_CATCH(PCOT_ERR_HOST)
}


}  // extern "C"
