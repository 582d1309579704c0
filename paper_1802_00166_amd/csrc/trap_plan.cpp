// Host planner of the concurrent-start trapezoid schedules (see trap.hpp).
#include <algorithm>
#include <cstdlib>
#include <vector>

#include "trap.hpp"

namespace pcot {

namespace {

struct Seg {
    int lo, hi, slo, shi, fo, v;
};

long long floor_div(long long a, long long b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// U and V segments covering the interior [1, n-1) of one dimension.  The
// natural pattern has U at [base + k P, base + k P + W) and V after it up to
// base + (k+1) P; a segment that reaches the array boundary is clipped there
// and that side gets slope 0 (the boundary cells never change).
std::vector<Seg> segments(int n, int F, int bt, int shift) {
    const long long W = F - 2, g = F - 2LL * bt, P = W + g;
    const long long base = 1 + shift;
    std::vector<Seg> out;
    for (long long k = floor_div(1 - base, P) - 1;; ++k) {
        const long long a = base + k * P;
        if (a >= n - 1) break;
        for (int v = 0; v < 2; ++v) {
            const long long lo = v ? a + W : a, hi = v ? a + P : a + W;
            if (hi <= 1 || lo >= n - 1) continue;
            Seg s;
            s.v = v;
            s.lo = (int)std::max<long long>(lo, 1);
            s.hi = (int)std::min<long long>(hi, n - 1);
            s.slo = lo <= 1 ? 0 : (v ? -1 : 1);
            s.shi = hi >= n - 1 ? 0 : (v ? 1 : -1);
            s.fo = (int)(v ? lo - bt : lo - 1);
            out.push_back(s);
        }
    }
    return out;
}

// Level-l range [a, b) of a segment (empty: a == b).
inline void lrange(const Seg& s, int l, int n, int& a, int& b) {
    a = std::max(s.lo + s.slo * l, 1);
    b = std::min(s.hi + s.shi * l, n - 1);
    if (b < a) b = a;
}

inline bool meets(int a0, int b0, int a1, int b1) { return a0 < b1 && a1 < b0 && a0 < b0 && a1 < b1; }

inline long long clip_len(int a, int b, int lo, int hi) {
    a = std::max(a, lo);
    b = std::min(b, hi);
    return b > a ? b - a : 0;
}

struct Band {
    std::vector<Seg> seg[2];
    int t0 = 0, nt = 0;
    std::vector<int> idx;  // queue index of tile (iy, ix), or -1
};

}  // namespace

TrapPlanHost build_trap_plan(int ny, int nx, int T, int bt, const int* F, bool shifted) {
    TrapPlanHost P;
    const int n[2] = {ny, nx};
    const int nb = (T + bt - 1) / bt;
    std::vector<Band> bands(nb);
    std::vector<std::pair<int, int>> edges;  // (pred, succ)
    std::vector<std::pair<int, int>> where;  // tile -> (iy, ix)
    for (int k = 0; k < nb; ++k) {
        Band& B = bands[k];
        B.t0 = k * bt;
        B.nt = std::min(bt, T - B.t0);
        for (int d = 0; d < 2; ++d) {
            const int half = F[d] - 1 - bt;  // half the period
            B.seg[d] = segments(n[d], F[d], bt, shifted && (k & 1) ? half : 0);
        }
        const int sy = (int)B.seg[0].size(), sx = (int)B.seg[1].size();
        B.idx.assign((size_t)sy * sx, -1);
        // queue: phases UU, UV, VU, VV, then row-major
        for (int vy = 0; vy < 2; ++vy)
            for (int vx = 0; vx < 2; ++vx)
                for (int iy = 0; iy < sy; ++iy) {
                    if (B.seg[0][iy].v != vy) continue;
                    for (int ix = 0; ix < sx; ++ix) {
                        if (B.seg[1][ix].v != vx) continue;
                        const Seg& Y = B.seg[0][iy];
                        const Seg& X = B.seg[1][ix];
                        TrapTile t;
                        t.lo[0] = Y.lo; t.hi[0] = Y.hi; t.slo[0] = Y.slo; t.shi[0] = Y.shi; t.fo[0] = Y.fo;
                        t.lo[1] = X.lo; t.hi[1] = X.hi; t.slo[1] = X.slo; t.shi[1] = X.shi; t.fo[1] = X.fo;
                        t.t0 = B.t0;
                        t.nt = B.nt;
                        t.need = 0;
                        t.succ0 = t.nsucc = 0;
                        t.pad = 0;
                        B.idx[(size_t)iy * sx + ix] = (int)P.tiles.size();
                        P.tiles.push_back(t);
                        where.emplace_back(iy, ix);
                    }
                }
        // same-band predecessors: a neighbour whose level l-1 range meets
        // this tile's level-l range grown by the stencil radius
        for (int iy = 0; iy < sy; ++iy)
            for (int ix = 0; ix < sx; ++ix) {
                const int me = B.idx[(size_t)iy * sx + ix];
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        const int jy = iy + dy, jx = ix + dx;
                        if ((dy == 0 && dx == 0) || jy < 0 || jy >= sy || jx < 0 || jx >= sx) continue;
                        const int other = B.idx[(size_t)jy * sx + jx];
                        bool dep = false;
                        for (int l = 1; l < B.nt && !dep; ++l) {
                            int a0, b0, a1, b1, c0, d0, c1, d1;
                            lrange(B.seg[0][iy], l, ny, a0, b0);
                            lrange(B.seg[0][jy], l - 1, ny, a1, b1);
                            lrange(B.seg[1][ix], l, nx, c0, d0);
                            lrange(B.seg[1][jx], l - 1, nx, c1, d1);
                            if (a0 == b0 || c0 == d0) continue;
                            dep = meets(a0 - 1, b0 + 1, a1, b1) && meets(c0 - 1, d0 + 1, c1, d1);
                        }
                        if (dep) edges.emplace_back(other, me);
                    }
            }
        // previous band: tiles whose top level meets this tile's level-0
        // range grown by the radius
        if (k > 0) {
            const Band& A = bands[k - 1];
            std::vector<std::vector<int>> hit[2];
            for (int d = 0; d < 2; ++d) {
                const int nn = n[d];
                hit[d].resize(B.seg[d].size());
                for (size_t i = 0; i < B.seg[d].size(); ++i) {
                    int a0, b0;
                    lrange(B.seg[d][i], 0, nn, a0, b0);
                    for (size_t j = 0; j < A.seg[d].size(); ++j) {
                        int a1, b1;
                        lrange(A.seg[d][j], A.nt - 1, nn, a1, b1);
                        if (meets(a0 - 1, b0 + 1, a1, b1)) hit[d][i].push_back((int)j);
                    }
                }
            }
            const int ax = (int)A.seg[1].size();
            for (int iy = 0; iy < sy; ++iy)
                for (int ix = 0; ix < sx; ++ix) {
                    const int me = B.idx[(size_t)iy * sx + ix];
                    for (int jy : hit[0][iy])
                        for (int jx : hit[1][ix]) {
                            const int other = A.idx[(size_t)jy * ax + jx];
                            if (other >= 0) edges.emplace_back(other, me);
                        }
                }
        }
    }
    // successor lists (CSR) and predecessor counts
    std::sort(edges.begin(), edges.end());
    edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
    P.succ.resize(edges.size());
    size_t e = 0;
    for (size_t q = 0; q < P.tiles.size(); ++q) {
        P.tiles[q].succ0 = (int)e;
        while (e < edges.size() && edges[e].first == (int)q) {
            P.succ[e] = edges[e].second;
            P.tiles[edges[e].second].need++;
            ++e;
        }
        P.tiles[q].nsucc = (int)e - P.tiles[q].succ0;
    }
    // algorithmic element transfers, as the executor performs them
    for (const TrapTile& t : P.tiles) {
        auto rng = [&](int d, int l, int& a, int& b) {
            a = std::max(t.lo[d] + t.slo[d] * l, 1);
            b = std::min(t.hi[d] + t.shi[d] * l, n[d] - 1);
            if (b < a) b = a;
        };
        int ya, yb, xa, xb;
        rng(0, 0, ya, yb);
        rng(1, 0, xa, xb);
        P.loads += clip_len(ya - 1, yb + 1, 0, ny) * clip_len(xa - 1, xb + 1, 0, nx);
        for (int l = 0; l < t.nt; ++l) {
            rng(0, l, ya, yb);
            rng(1, l, xa, xb);
            if (ya == yb || xa == xb) continue;
            if (l > 0) {
                const long long wx = clip_len(xa - 1, xb + 1, 0, nx), hy = clip_len(ya - 1, yb + 1, 0, ny);
                P.loads += 2 * wx * ((t.slo[0] < 0) + (t.shi[0] > 0));
                P.loads += 2 * hy * ((t.slo[1] < 0) + (t.shi[1] > 0));
            }
            if (l == t.nt - 1) {
                P.stores += (long long)(yb - ya) * (xb - xa);
            } else {
                const long long h = yb - ya, w = xb - xa;
                P.stores += std::min<long long>(2, h) * w * ((t.slo[0] > 0) + (t.shi[0] < 0));
                P.stores += std::min<long long>(2, w) * h * ((t.slo[1] > 0) + (t.shi[1] < 0));
            }
        }
    }
    return P;
}

}  // namespace pcot
