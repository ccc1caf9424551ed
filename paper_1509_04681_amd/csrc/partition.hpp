// partition.hpp -- balanced k-way graph partitioning by recursive bisection,
// for the column blocks of the block-wise method: Sec. 4.1 clusters the
// active set of Lambda so that few active entries fall in off-diagonal
// blocks (each such block costs a recomputation of Sigma and Psi columns),
// and Sec. 4.2 clusters the columns of Theta through the graph of
// Theta^T Theta so that a row's active entries fall in few column blocks.
// Both minimise the edge cut of a graph under a bound on the block size.
// Host C++ only (no HIP), so it is also built and tested with g++ under the
// sanitizers.
//
// Each bisection is multilevel: the graph is coarsened by heavy-edge
// matching, split on the coarsest level by greedy growing from several
// seeds (always adding the frontier vertex with the heaviest connection into
// the growing side), and the split is projected back level by level and
// improved by Fiduccia-Mattheyses passes (vertices move one at a time, the
// best-gain move that keeps both sides feasible first, each vertex at most
// once per pass, the pass rolled back to its best prefix).  The size bounds
// of a bisection are exactly those under which both sides can still be
// split into their parts with every part within the limit, so the final
// parts always respect it.  Deterministic.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <queue>
#include <utility>
#include <vector>

namespace cggm {
namespace part {

// Undirected simple graph in CSR (both directions listed, no self loops,
// sorted neighbour lists).
struct Graph {
    int64_t n = 0;
    std::vector<int64_t> ptr;   // n + 1
    std::vector<int32_t> adj;
};

// The union of the listed entries (u, v) and (v, u) of a CSR pattern, self
// loops and repeats dropped.  Returns false when the pattern is malformed
// (rowptr not starting at 0 or decreasing, a column outside [0, n)).
inline bool undirected(int64_t n, const int64_t *rowptr, const int32_t *col, Graph &g) {
    if (n < 0 || rowptr[0] != 0) return false;
    for (int64_t i = 0; i < n; ++i)
        if (rowptr[i + 1] < rowptr[i]) return false;
    std::vector<int64_t> deg(n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t t = rowptr[i]; t < rowptr[i + 1]; ++t) {
            const int64_t j = col[t];
            if (j < 0 || j >= n) return false;
            if (j == i) continue;
            ++deg[i + 1];
            ++deg[j + 1];
        }
    std::vector<int64_t> start(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) start[i + 1] = start[i] + deg[i + 1];
    std::vector<int32_t> raw(start[n]);
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t t = rowptr[i]; t < rowptr[i + 1]; ++t) {
            const int64_t j = col[t];
            if (j == i) continue;
            raw[fill[i]++] = (int32_t)j;
            raw[fill[j]++] = (int32_t)i;
        }
    g.n = n;
    g.ptr.assign(n + 1, 0);
    g.adj.clear();
    g.adj.reserve(raw.size());
    for (int64_t i = 0; i < n; ++i) {
        std::sort(raw.begin() + start[i], raw.begin() + start[i + 1]);
        const auto e = std::unique(raw.begin() + start[i], raw.begin() + start[i + 1]);
        g.adj.insert(g.adj.end(), raw.begin() + start[i], e);
        g.ptr[i + 1] = (int64_t)g.adj.size();
    }
    return true;
}

// Number of undirected edges whose ends lie in different parts.
inline int64_t edge_cut(const Graph &g, const int32_t *part) {
    int64_t cut = 0;
    for (int64_t v = 0; v < g.n; ++v)
        for (int64_t t = g.ptr[v]; t < g.ptr[v + 1]; ++t)
            if (g.adj[t] > v && part[g.adj[t]] != part[v]) ++cut;
    return cut;
}

// Weighted graph of one bisection: vertex weights (vertices merged by
// coarsening) and edge weights (edges merged), CSR with both directions.
struct WGraph {
    int64_t n = 0;
    std::vector<int64_t> ptr, ew, vw;
    std::vector<int32_t> adj;
    int64_t total() const {
        int64_t t = 0;
        for (int64_t w : vw) t += w;
        return t;
    }
};

// The subgraph induced by the vertices vs (global indices), unit weights.
inline WGraph induced(const Graph &g, const std::vector<int32_t> &vs, std::vector<int32_t> &loc) {
    WGraph w;
    w.n = (int64_t)vs.size();
    for (int64_t k = 0; k < w.n; ++k) loc[vs[k]] = (int32_t)k;
    w.ptr.assign(w.n + 1, 0);
    for (int64_t k = 0; k < w.n; ++k) {
        const int32_t v = vs[k];
        for (int64_t t = g.ptr[v]; t < g.ptr[v + 1]; ++t)
            if (loc[g.adj[t]] >= 0) {
                w.adj.push_back(loc[g.adj[t]]);
                w.ew.push_back(1);
            }
        w.ptr[k + 1] = (int64_t)w.adj.size();
    }
    w.vw.assign(w.n, 1);
    for (int32_t v : vs) loc[v] = -1;
    return w;
}

// A fixed scrambling of the vertex order (splitmix64 of the index), so that
// the matching visits vertices in no structured order yet repeats exactly.
inline uint64_t mix64(uint64_t x) {
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

// One coarsening step by heavy-edge matching: each vertex, in the scrambled
// order, is merged with its unmatched neighbour of the heaviest connecting
// edge (ties: the lowest index) if their weights together stay within
// max_vw.  Returns false when it would shrink the graph by less than 10%.
inline bool coarsen(const WGraph &f, WGraph &c, std::vector<int32_t> &map, int64_t max_vw) {
    const int64_t n = f.n;
    std::vector<std::pair<uint64_t, int32_t>> order(n);
    for (int64_t v = 0; v < n; ++v) order[v] = {mix64((uint64_t)v), (int32_t)v};
    std::sort(order.begin(), order.end());
    std::vector<int32_t> mate(n, -1);
    for (const auto &o : order) {
        const int32_t v = o.second;
        if (mate[v] >= 0) continue;
        int32_t best = v;
        int64_t bw = -1;
        for (int64_t t = f.ptr[v]; t < f.ptr[v + 1]; ++t) {
            const int32_t u = f.adj[t];
            if (mate[u] >= 0 || u == v || f.vw[u] + f.vw[v] > max_vw) continue;
            if (f.ew[t] > bw || (f.ew[t] == bw && u < best)) {
                bw = f.ew[t];
                best = u;
            }
        }
        mate[v] = best;
        mate[best] = v;
    }
    map.assign(n, -1);
    int64_t nc = 0;
    for (int64_t v = 0; v < n; ++v)
        if (map[v] < 0) {
            map[v] = (int32_t)nc;
            map[mate[v]] = (int32_t)nc;
            ++nc;
        }
    if (nc > n - n / 10) return false;
    c.n = nc;
    c.vw.assign(nc, 0);
    for (int64_t v = 0; v < n; ++v) c.vw[map[v]] += f.vw[v];
    // merge the neighbour lists of each coarse vertex, summing edge weights
    std::vector<std::vector<int32_t>> members(nc);
    for (int64_t v = 0; v < n; ++v) members[map[v]].push_back((int32_t)v);
    std::vector<int64_t> acc(nc, 0);
    std::vector<int32_t> touched;
    c.ptr.assign(nc + 1, 0);
    for (int64_t cv = 0; cv < nc; ++cv) {
        touched.clear();
        for (int32_t v : members[cv])
            for (int64_t t = f.ptr[v]; t < f.ptr[v + 1]; ++t) {
                const int32_t cu = map[f.adj[t]];
                if (cu == cv) continue;
                if (acc[cu] == 0) touched.push_back(cu);
                acc[cu] += f.ew[t];
            }
        std::sort(touched.begin(), touched.end());
        for (int32_t cu : touched) {
            c.adj.push_back(cu);
            c.ew.push_back(acc[cu]);
            acc[cu] = 0;
        }
        c.ptr[cv + 1] = (int64_t)c.adj.size();
    }
    return true;
}

inline int64_t wcut(const WGraph &g, const std::vector<uint8_t> &side) {
    int64_t cut = 0;
    for (int64_t v = 0; v < g.n; ++v)
        for (int64_t t = g.ptr[v]; t < g.ptr[v + 1]; ++t)
            if (side[g.adj[t]] != side[v]) cut += g.ew[t];
    return cut / 2;
}

// The vertex BFS reaches last from `s` inside its component (ties: the
// lowest index).
inline int32_t far_from(const WGraph &g, int32_t s) {
    std::vector<int32_t> dist(g.n, -1), q{s};
    dist[s] = 0;
    int32_t last = s;
    for (size_t h = 0; h < q.size(); ++h) {
        const int32_t v = q[h];
        if (dist[v] > dist[last] || (dist[v] == dist[last] && v < last)) last = v;
        for (int64_t t = g.ptr[v]; t < g.ptr[v + 1]; ++t)
            if (dist[g.adj[t]] < 0) {
                dist[g.adj[t]] = dist[v] + 1;
                q.push_back(g.adj[t]);
            }
    }
    return last;
}

// Side 0 grown from `seed` until its weight reaches `target`: always the
// frontier vertex with the heaviest connection into side 0 (ties: the lowest
// index); a new seed (peripheral in its component) when a component is
// exhausted.
inline void grow(const WGraph &g, int32_t seed, int64_t target, std::vector<uint8_t> &side) {
    side.assign(g.n, 1);
    std::vector<int64_t> inside(g.n, 0);
    std::priority_queue<std::pair<int64_t, int32_t>> heap;
    int64_t size = 0;
    int32_t next_seed = 0;
    int32_t pick = seed;
    while (size < target) {
        if (pick < 0) {
            while (!heap.empty()) {
                const auto top = heap.top();
                heap.pop();
                const int32_t u = -top.second;
                if (side[u] == 1 && top.first == inside[u]) {
                    pick = u;
                    break;
                }
            }
        }
        if (pick < 0) {
            while (next_seed < g.n && side[next_seed] == 0) ++next_seed;
            if (next_seed >= g.n) break;
            pick = far_from(g, far_from(g, next_seed));
        }
        side[pick] = 0;
        size += g.vw[pick];
        for (int64_t t = g.ptr[pick]; t < g.ptr[pick + 1]; ++t) {
            const int32_t u = g.adj[t];
            if (side[u] == 1) {
                inside[u] += g.ew[t];
                heap.push({inside[u], -u});
            }
        }
        pick = -1;
    }
}

// Moves vertices of best gain off the heavier side until the weight of side
// 0 lies in [lo, hi] (a vertex that would overshoot the other bound is
// passed over; stops when none can move).
inline void rebalance(const WGraph &g, std::vector<uint8_t> &side, int64_t lo, int64_t hi) {
    int64_t size0 = 0;
    for (int64_t v = 0; v < g.n; ++v) size0 += side[v] == 0 ? g.vw[v] : 0;
    if (size0 >= lo && size0 <= hi) return;
    const int from = size0 > hi ? 0 : 1;
    std::vector<int64_t> gain(g.n, 0);
    std::priority_queue<std::pair<int64_t, int32_t>> heap;
    for (int32_t v = 0; v < g.n; ++v) {
        for (int64_t t = g.ptr[v]; t < g.ptr[v + 1]; ++t)
            gain[v] += side[g.adj[t]] != side[v] ? g.ew[t] : -g.ew[t];
        if (side[v] == from) heap.push({gain[v], -v});
    }
    while ((from == 0 && size0 > hi) || (from == 1 && size0 < lo)) {
        int32_t v = -1;
        while (!heap.empty()) {
            const auto e = heap.top();
            heap.pop();
            const int32_t u = -e.second;
            if (side[u] != from || e.first != gain[u]) continue;
            const int64_t ns = from == 0 ? size0 - g.vw[u] : size0 + g.vw[u];
            if ((from == 0 && ns < lo) || (from == 1 && ns > hi)) continue;
            v = u;
            break;
        }
        if (v < 0) return;
        side[v] = (uint8_t)(1 - from);
        size0 += from == 0 ? -g.vw[v] : g.vw[v];
        gain[v] = -gain[v];
        for (int64_t t = g.ptr[v]; t < g.ptr[v + 1]; ++t) {
            const int32_t u = g.adj[t];
            gain[u] += side[u] == side[v] ? -2 * g.ew[t] : 2 * g.ew[t];
            if (side[u] == from) heap.push({gain[u], -u});
        }
    }
}

// One Fiduccia-Mattheyses pass: the best-gain vertex of either side moves
// (each vertex at most once) as long as the weight of side 0 stays within
// the heaviest vertex of [lo, hi], and the pass is rolled back to its best
// prefix among the states with that weight in [lo, hi].  True when it
// lowered the cut (or first reached a balanced state).
inline bool fm_pass(const WGraph &g, std::vector<uint8_t> &side, int64_t lo, int64_t hi) {
    const int64_t m = g.n;
    std::vector<int64_t> gain(m, 0);
    int64_t size0 = 0, tol = 1;
    for (int32_t v = 0; v < m; ++v) {
        for (int64_t t = g.ptr[v]; t < g.ptr[v + 1]; ++t)
            gain[v] += side[g.adj[t]] != side[v] ? g.ew[t] : -g.ew[t];
        size0 += side[v] == 0 ? g.vw[v] : 0;
        tol = std::max(tol, g.vw[v]);
    }
    const bool init_ok = size0 >= lo && size0 <= hi;
    std::priority_queue<std::pair<int64_t, int32_t>> heap[2];
    for (int32_t v = 0; v < m; ++v) heap[side[v]].push({gain[v], -v});
    std::vector<uint8_t> locked(m, 0);
    std::vector<int32_t> moved;
    int64_t total = 0, best = 0;
    bool found = init_ok;
    size_t best_len = 0;
    const size_t patience = 64 + (size_t)m / 16;
    auto top_of = [&](int s) -> int32_t {
        while (!heap[s].empty()) {
            const auto e = heap[s].top();
            const int32_t v = -e.second;
            if (!locked[v] && side[v] == s && e.first == gain[v]) return v;
            heap[s].pop();
        }
        return -1;
    };
    while (true) {
        int32_t a = top_of(0), b = top_of(1);
        if (a >= 0 && size0 - g.vw[a] < lo - tol) a = -1;   // 0 -> 1: side 0 too light
        if (b >= 0 && size0 + g.vw[b] > hi + tol) b = -1;   // 1 -> 0: side 0 too heavy
        int32_t v;
        if (a < 0 && b < 0) break;
        if (a < 0) v = b;
        else if (b < 0) v = a;
        else v = (gain[a] > gain[b] || (gain[a] == gain[b] && a < b)) ? a : b;
        const int s = side[v];
        heap[s].pop();
        locked[v] = 1;
        side[v] = (uint8_t)(1 - s);
        size0 += s == 0 ? -g.vw[v] : g.vw[v];
        total += gain[v];
        moved.push_back(v);
        gain[v] = -gain[v];
        for (int64_t t = g.ptr[v]; t < g.ptr[v + 1]; ++t) {
            const int32_t u = g.adj[t];
            // the edge became uncut for u on v's new side, cut otherwise
            gain[u] += side[u] == side[v] ? -2 * g.ew[t] : 2 * g.ew[t];
            if (!locked[u]) heap[side[u]].push({gain[u], -u});
        }
        if (size0 >= lo && size0 <= hi && (!found || total > best)) {
            best = total;
            best_len = moved.size();
            found = true;
        } else if (moved.size() - best_len > patience) {
            break;
        }
    }
    for (size_t k = moved.size(); k > best_len; --k) side[moved[k - 1]] ^= 1;
    return best_len > 0 && (best > 0 || !init_ok);
}

inline void refine(const WGraph &g, std::vector<uint8_t> &side, int64_t lo, int64_t hi) {
    rebalance(g, side, lo, hi);
    for (int pass = 0; pass < 10; ++pass)
        if (!fm_pass(g, side, lo, hi)) break;
}

// Multilevel bisection of the unit-weight graph g0 with the weight of side 0
// in [lo, hi] (aiming at `target`): heavy-edge matching down to a few dozen
// vertices, four greedy growths from different seeds refined there (the
// best cut kept), then projection and refinement level by level; the size
// bounds are relaxed by the heaviest vertex on the coarse levels and exact
// on the finest.
inline std::vector<uint8_t> bisect(const WGraph &g0, int64_t lo, int64_t hi, int64_t target) {
    std::vector<WGraph> levels;
    std::vector<std::vector<int32_t>> maps;
    levels.push_back(g0);
    const int64_t max_vw = std::max<int64_t>(1, g0.total() / 40);
    while (levels.back().n > 64 && levels.size() < 40) {
        WGraph c;
        std::vector<int32_t> map;
        if (!coarsen(levels.back(), c, map, max_vw)) break;
        maps.push_back(std::move(map));
        levels.push_back(std::move(c));
    }
    auto slack = [&](const WGraph &g) {
        int64_t w = 0;
        for (int64_t x : g.vw) w = std::max(w, x);
        return w - 1;
    };
    const WGraph &cg = levels.back();
    const int64_t sc = slack(cg);
    std::vector<uint8_t> side, best_side;
    int64_t best_cut = -1;
    const int32_t seeds[4] = {far_from(cg, far_from(cg, 0)), (int32_t)(cg.n / 4),
                              (int32_t)(cg.n / 2), (int32_t)(3 * cg.n / 4)};
    for (int32_t seed : seeds) {
        grow(cg, seed, target, side);
        refine(cg, side, lo - sc, hi + sc);
        const int64_t c = wcut(cg, side);
        if (best_cut < 0 || c < best_cut) {
            best_cut = c;
            best_side = side;
        }
    }
    side = best_side;
    for (size_t l = levels.size() - 1; l > 0; --l) {
        const WGraph &f = levels[l - 1];
        std::vector<uint8_t> fs(f.n);
        for (int64_t v = 0; v < f.n; ++v) fs[v] = side[maps[l - 1][v]];
        const int64_t s = l - 1 == 0 ? 0 : slack(f);
        refine(f, fs, lo - s, hi + s);
        side.swap(fs);
    }
    if (levels.size() == 1) refine(g0, side, lo, hi);
    return side;
}

// Parts [p0, p0 + k) for the vertices vs (global indices), every part with
// at least one and at most `cap` vertices.
inline void recurse(const Graph &g, const std::vector<int32_t> &vs, int32_t p0, int64_t k,
                    int64_t cap, double imbalance, std::vector<int32_t> &loc, int32_t *part) {
    const int64_t m = (int64_t)vs.size();
    if (k == 1) {
        for (int32_t v : vs) part[v] = p0;
        return;
    }
    const int64_t kl = k / 2, kr = k - kl;
    const int64_t lo = std::max(kl, m - kr * cap), hi = std::min(m - kr, kl * cap);
    const int64_t target = std::min(hi, std::max(lo, (m * kl + k / 2) / k));
    // each of the ceil(log2 k) levels of bisections below takes an equal
    // share of the allowed imbalance, so the first splits do not spend it all
    int levels = 0;
    while ((int64_t(1) << levels) < k) ++levels;
    const double eps = std::pow(1.0 + imbalance, 1.0 / levels) - 1.0;
    const int64_t lo2 = std::max(lo, (int64_t)std::floor((double)target * (1.0 - eps)));
    const int64_t hi2 = std::min(hi, (int64_t)std::ceil((double)target * (1.0 + eps)));
    const std::vector<uint8_t> side = bisect(induced(g, vs, loc), lo2, hi2, target);
    std::vector<int32_t> left, right;
    for (int64_t t = 0; t < m; ++t) (side[t] == 0 ? left : right).push_back(vs[t]);
    recurse(g, left, p0, kl, cap, imbalance, loc, part);
    recurse(g, right, p0 + (int32_t)kl, kr, cap, imbalance, loc, part);
}

// Largest part size allowed: (1 + imbalance) times the mean, rounded down,
// and at least the mean rounded up.
inline int64_t part_cap(int64_t n, int64_t k, double imbalance) {
    const int64_t mean_up = (n + k - 1) / k;
    const double c = (1.0 + imbalance) * (double)n / (double)k;
    return std::max<int64_t>(mean_up, (int64_t)c);
}

inline void partition(const Graph &g, int64_t k, double imbalance, int32_t *part) {
    std::vector<int32_t> all(g.n);
    for (int64_t v = 0; v < g.n; ++v) all[v] = (int32_t)v;
    std::vector<int32_t> loc(g.n, -1);   // global -> local index of a bisection's vertices
    recurse(g, all, 0, k, part_cap(g.n, k, imbalance), imbalance, loc, part);
}

}  // namespace part
}  // namespace cggm
