// Host planner: leaf enumeration and visiting orders (see plan.hpp).
#include "plan.hpp"

#include <algorithm>
#include <unordered_map>

namespace pcot {

StencilGeom make_geom(int d, const int64_t* dims, int64_t T, const int64_t* tile) {
    StencilGeom g;
    g.d = d;
    g.T = T;
    for (int i = 0; i < d; ++i) g.n[i] = dims[i];
    for (int i = 0; i <= d; ++i) g.b[i] = tile[i];
    g.cnt[0] = (T + g.b[0] - 1) / g.b[0];
    for (int i = 0; i < d; ++i) {
        const int64_t extent = g.n[i] - 2 + T - 1;  // j in [1, n-2+T-1]
        g.cnt[i + 1] = (extent + g.b[i + 1] - 1) / g.b[i + 1];
    }
    return g;
}

// The time range over which every spatial interval of the box meets the
// shifting domain interval [1 + t, n - 2 + t]:
//   lo_k <= n_k - 2 + t  and  lo_k + size_k - 1 >= 1 + t.
bool box_nonempty(const StencilGeom& g, const int64_t* lo, const int64_t* size) {
    for (int i = 0; i <= g.d; ++i)
        if (size[i] <= 0) return false;
    int64_t tmin = std::max<int64_t>(lo[0], 0);
    int64_t tmax = std::min<int64_t>(lo[0] + size[0] - 1, g.T - 1);
    for (int k = 0; k < g.d; ++k) {
        tmin = std::max<int64_t>(tmin, lo[k + 1] - g.n[k] + 2);
        tmax = std::min<int64_t>(tmax, lo[k + 1] + size[k + 1] - 2);
    }
    return tmin <= tmax;
}

bool leaf_nonempty(const StencilGeom& g, const int32_t* k) {
    int64_t lo[4], sz[4];
    for (int i = 0; i <= g.d; ++i) {
        if (k[i] < 0 || k[i] >= g.cnt[i]) return false;
        lo[i] = (i == 0 ? 0 : 1) + (int64_t)k[i] * g.b[i];
        sz[i] = g.b[i];
    }
    return box_nonempty(g, lo, sz);
}

int count_preds(const StencilGeom& g, const int32_t* k) {
    const int D = g.d + 1;
    int c = 0;
    for (int m = 1; m < (1 << D); ++m) {
        int32_t q[4] = {0, 0, 0, 0};
        for (int i = 0; i < D; ++i) q[i] = k[i] - ((m >> (D - 1 - i)) & 1);
        if (leaf_nonempty(g, q)) ++c;
    }
    return c;
}

namespace {

void slt(const StencilGeom& g, std::vector<Leaf>& out) {
    const int D = g.d + 1;
    int32_t k[4] = {0, 0, 0, 0};
    // lexicographic: time outermost, innermost spatial last
    int64_t total = 1;
    for (int i = 0; i < D; ++i) total *= g.cnt[i];
    for (int64_t idx = 0; idx < total; ++idx) {
        int64_t r = idx;
        for (int i = D - 1; i >= 0; --i) {
            k[i] = (int32_t)(r % g.cnt[i]);
            r /= g.cnt[i];
        }
        if (leaf_nonempty(g, k)) {
            Leaf L;
            for (int i = 0; i < 4; ++i) L.k[i] = i < D ? k[i] : 0;
            out.push_back(L);
        }
    }
}

// Recursive decomposition of the padded bounding box.  An orthant larger than
// the leaf in some dimension is halved there; in dimensions already at leaf
// size the second half has zero width and is skipped (zero-orthant exit);
// orthants without a domain point are skipped (empty-orthant exit).
// Sequential: orthants in lexicographic order.  Grouped (the parallel
// version): orthants with the same number of upper halves form one group of
// concurrent tasks, groups are separated by a taskwait; a group's concurrent
// execution is serialised into the queue by merging its members' leaf
// sequences round-robin.
void cot_rec(const StencilGeom& g, const int64_t* org, const int64_t* sz, bool grouped,
             std::vector<Leaf>& out) {
    const int D = g.d + 1;
    if (!box_nonempty(g, org, sz)) return;
    bool leaf = true;
    for (int i = 0; i < D; ++i)
        if (sz[i] > g.b[i]) leaf = false;
    if (leaf) {
        Leaf L = {{0, 0, 0, 0}};
        for (int i = 0; i < D; ++i) L.k[i] = (int32_t)((org[i] - (i == 0 ? 0 : 1)) / g.b[i]);
        out.push_back(L);
        return;
    }
    int64_t h[4][2][2];  // [dim][half] -> {origin, size}
    for (int i = 0; i < D; ++i) {
        if (sz[i] > g.b[i]) {
            const int64_t half = sz[i] / 2;
            h[i][0][0] = org[i];        h[i][0][1] = half;
            h[i][1][0] = org[i] + half; h[i][1][1] = sz[i] - half;
        } else {
            h[i][0][0] = org[i];         h[i][0][1] = sz[i];
            h[i][1][0] = org[i] + sz[i]; h[i][1][1] = 0;
        }
    }
    const int nch = 1 << D;  // bit D-1-i of a child index = half of dim i
    auto child = [&](int m, std::vector<Leaf>& dst) {
        int64_t o2[4], s2[4];
        for (int i = 0; i < D; ++i) {
            const int bit = (m >> (D - 1 - i)) & 1;
            o2[i] = h[i][bit][0];
            s2[i] = h[i][bit][1];
            if (s2[i] == 0) return;  // zero orthant
        }
        cot_rec(g, o2, s2, grouped, dst);
    };
    if (!grouped) {
        for (int m = 0; m < nch; ++m) child(m, out);
        return;
    }
    for (int grp = 0; grp <= D; ++grp) {
        std::vector<std::vector<Leaf>> seqs;
        size_t longest = 0;
        for (int m = 0; m < nch; ++m) {
            if (__builtin_popcount(m) != grp) continue;
            seqs.emplace_back();
            child(m, seqs.back());
            longest = std::max(longest, seqs.back().size());
        }
        for (size_t i = 0; i < longest; ++i)
            for (auto& q : seqs)
                if (i < q.size()) out.push_back(q[i]);
    }
}

}  // namespace

std::vector<Leaf> enumerate_leaves(const StencilGeom& g, int schedule) {
    std::vector<Leaf> out;
    const int D = g.d + 1;
    if (schedule == 1 || schedule == 2) {
        slt(g, out);
        if (schedule == 2) {
            std::stable_sort(out.begin(), out.end(), [D](const Leaf& a, const Leaf& b) {
                int64_t sa = 0, sb = 0;
                for (int i = 0; i < D; ++i) { sa += a.k[i]; sb += b.k[i]; }
                return sa < sb;
            });
        }
    } else {
        int64_t org[4], sz[4];
        for (int i = 0; i < D; ++i) {
            org[i] = i == 0 ? 0 : 1;
            const int64_t extent = i == 0 ? g.T : g.n[i - 1] - 2 + g.T - 1;
            int64_t e = g.b[i];
            while (e < extent) e *= 2;  // smallest b * 2^k >= extent
            sz[i] = e;
        }
        cot_rec(g, org, sz, schedule == 4, out);
    }
    return out;
}

std::string check_order(const StencilGeom& g, const std::vector<Leaf>& order) {
    const int D = g.d + 1;
    auto key = [&](const int32_t* k) {
        int64_t v = 0;
        for (int i = 0; i < D; ++i) v = v * g.cnt[i] + k[i];
        return v;
    };
    std::unordered_map<int64_t, int64_t> pos;
    pos.reserve(order.size() * 2);
    for (size_t i = 0; i < order.size(); ++i) {
        if (!leaf_nonempty(g, order[i].k)) return "empty leaf in order";
        if (!pos.emplace(key(order[i].k), (int64_t)i).second) return "duplicate leaf";
    }
    int64_t total = 1, nonempty = 0;
    for (int i = 0; i < D; ++i) total *= g.cnt[i];
    int32_t k[4] = {0, 0, 0, 0};
    for (int64_t idx = 0; idx < total; ++idx) {
        int64_t r = idx;
        for (int i = D - 1; i >= 0; --i) { k[i] = (int32_t)(r % g.cnt[i]); r /= g.cnt[i]; }
        if (!leaf_nonempty(g, k)) continue;
        ++nonempty;
        auto it = pos.find(key(k));
        if (it == pos.end()) return "non-empty leaf missing from order";
        for (int m = 1; m < (1 << D); ++m) {
            int32_t q[4] = {0, 0, 0, 0};
            for (int i = 0; i < D; ++i) q[i] = k[i] - ((m >> (D - 1 - i)) & 1);
            if (!leaf_nonempty(g, q)) continue;
            auto jt = pos.find(key(q));
            if (jt == pos.end() || jt->second >= it->second) return "predecessor not before successor";
        }
    }
    if (nonempty != (int64_t)order.size()) return "leaf count mismatch";
    return "";
}

}  // namespace pcot
