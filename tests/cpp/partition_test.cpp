// Host test of the graph partitioner (paper_1509_04681_amd/csrc/partition.hpp),
// built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer:
// validity of every partition (all vertices placed, part sizes within the
// bound, the reported cut equal to a recount), optimal cuts where they are
// known (paths, disjoint cliques, graphs without edges), malformed patterns
// rejected, and determinism.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <random>
#include <set>
#include <utility>
#include <vector>

#include "partition.hpp"

using namespace cggm::part;

static int failures = 0;
#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                            \
        }                                                          \
    } while (0)

struct Csr {
    std::vector<int64_t> ptr;
    std::vector<int32_t> col;
};

// Upper-triangle listing of an undirected edge set (the partitioner takes
// the union with the transposed pairs).
static Csr from_edges(int64_t n, const std::vector<std::pair<int, int>> &edges) {
    std::vector<std::vector<int32_t>> rows(n);
    for (auto e : edges) rows[std::min(e.first, e.second)].push_back(std::max(e.first, e.second));
    Csr c;
    c.ptr.push_back(0);
    for (auto &r : rows) {
        c.col.insert(c.col.end(), r.begin(), r.end());
        c.ptr.push_back((int64_t)c.col.size());
    }
    return c;
}

static int64_t recount(int64_t n, const std::vector<std::pair<int, int>> &edges,
                       const std::vector<int32_t> &part) {
    std::set<std::pair<int, int>> uniq;
    for (auto e : edges)
        if (e.first != e.second)
            uniq.insert({std::min(e.first, e.second), std::max(e.first, e.second)});
    int64_t cut = 0;
    for (auto e : uniq) cut += part[e.first] != part[e.second];
    (void)n;
    return cut;
}

// Partitions and checks validity; returns the cut.
static int64_t run(int64_t n, const std::vector<std::pair<int, int>> &edges, int64_t k,
                   double imb, std::vector<int32_t> &part) {
    Csr c = from_edges(n, edges);
    Graph g;
    CHECK(undirected(n, c.ptr.data(), c.col.data(), g));
    part.assign(n, -1);
    partition(g, k, imb, part.data());
    const int64_t cap = part_cap(n, k, imb);
    std::vector<int64_t> size(k, 0);
    for (int64_t v = 0; v < n; ++v) {
        CHECK(part[v] >= 0 && part[v] < k);
        if (part[v] >= 0 && part[v] < k) ++size[part[v]];
    }
    for (int64_t p = 0; p < k; ++p) CHECK(size[p] >= 1 && size[p] <= cap);
    const int64_t cut = edge_cut(g, part.data());
    CHECK(cut == recount(n, edges, part));
    return cut;
}

int main() {
    std::vector<int32_t> part;
    // paths: k - 1 cut edges, exact sizes when k divides n
    {
        std::vector<std::pair<int, int>> e;
        for (int i = 0; i + 1 < 1000; ++i) e.push_back({i, i + 1});
        CHECK(run(1000, e, 8, 0.0, part) == 7);
        std::vector<int> cnt(8, 0);
        for (int v = 0; v < 1000; ++v) ++cnt[part[v]];
        for (int p = 0; p < 8; ++p) CHECK(cnt[p] == 125);
        CHECK(run(1000, e, 1, 0.0, part) == 0);
        CHECK(run(1000, e, 3, 0.05, part) == 2);
        // a path listed in shuffled order with both directions and repeats
        std::vector<std::pair<int, int>> e2 = e;
        for (auto x : e) e2.push_back({x.second, x.first});
        std::mt19937 rng(5);
        std::shuffle(e2.begin(), e2.end(), rng);
        CHECK(run(1000, e2, 8, 0.0, part) == 7);
    }
    // disjoint cliques under a random relabelling: recovered exactly
    {
        const int nc = 8, cs = 50, n = nc * cs;
        std::vector<int> perm(n);
        for (int i = 0; i < n; ++i) perm[i] = i;
        std::mt19937 rng(7);
        std::shuffle(perm.begin(), perm.end(), rng);
        std::vector<std::pair<int, int>> e;
        for (int c = 0; c < nc; ++c)
            for (int a = 0; a < cs; ++a)
                for (int b = a + 1; b < cs; ++b) e.push_back({perm[c * cs + a], perm[c * cs + b]});
        CHECK(run(n, e, nc, 0.0, part) == 0);
        CHECK(run(n, e, 4, 0.0, part) == 0);
    }
    // no edges; one vertex per part; a ragged bound
    {
        std::vector<std::pair<int, int>> none;
        CHECK(run(10, none, 3, 0.0, part) == 0);
        CHECK(run(10, none, 10, 0.0, part) == 0);
        std::vector<std::pair<int, int>> e;
        for (int i = 0; i + 1 < 37; ++i) e.push_back({i, i + 1});
        CHECK(run(37, e, 37, 0.0, part) == 36);
        CHECK(run(37, e, 5, 0.0, part) == 4);
    }
    // random graph: validity, determinism, and a cut well below a random
    // balanced assignment's
    {
        const int n = 3000;
        std::mt19937 rng(11);
        std::uniform_int_distribution<int> U(0, n - 1);
        std::vector<std::pair<int, int>> e;
        for (int t = 0; t < 4 * n; ++t) e.push_back({U(rng), U(rng)});
        std::vector<int32_t> p1, p2;
        const int64_t c1 = run(n, e, 16, 0.03, p1);
        const int64_t c2 = run(n, e, 16, 0.03, p2);
        CHECK(c1 == c2 && p1 == p2);
        std::vector<int32_t> rnd(n);
        for (int v = 0; v < n; ++v) rnd[v] = v % 16;
        CHECK(c1 < recount(n, e, rnd) * 2 / 3);
        printf("random graph n=%d m=%zu k=16: cut %lld (round robin %lld)\n", n, e.size(),
               (long long)c1, (long long)recount(n, e, rnd));
    }
    // grid 40 x 40 into 4: the straight cuts give 80, the optimum
    {
        const int w = 40;
        std::vector<std::pair<int, int>> e;
        for (int r = 0; r < w; ++r)
            for (int c = 0; c < w; ++c) {
                if (c + 1 < w) e.push_back({r * w + c, r * w + c + 1});
                if (r + 1 < w) e.push_back({r * w + c, (r + 1) * w + c});
            }
        const int64_t cut = run(w * w, e, 4, 0.03, part);
        printf("grid %dx%d k=4: cut %lld\n", w, w, (long long)cut);
        CHECK(cut == 80);
    }
    // random small graphs of every shape: sizes from 1, k from 1 to n,
    // densities from empty to dense, several components, repeats and self
    // loops; every partition valid (checked inside run) and repeatable
    {
        std::mt19937 rng(2024);
        for (int trial = 0; trial < 250; ++trial) {
            const int n = 1 + (int)(rng() % 160);
            const int k = 1 + (int)(rng() % n);
            const double dens[4] = {0.0, 0.01, 0.05, 0.4};
            const double dp = dens[rng() % 4];
            const double imbs[3] = {0.0, 0.03, 0.25};
            const double imb = imbs[rng() % 3];
            std::bernoulli_distribution coin(dp);
            std::vector<std::pair<int, int>> e;
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b)
                    if (coin(rng)) e.push_back({a, b});   // both orders, self loops
            std::vector<int32_t> p1, p2;
            const int64_t c1 = run(n, e, k, imb, p1);
            const int64_t c2 = run(n, e, k, imb, p2);
            CHECK(c1 == c2 && p1 == p2);
        }
    }
    // malformed patterns
    {
        Graph g;
        std::vector<int64_t> ptr = {0, 2, 1, 3};
        std::vector<int32_t> col = {1, 2, 0};
        CHECK(!undirected(3, ptr.data(), col.data(), g));
        std::vector<int64_t> ptr2 = {0, 1, 2, 3};
        std::vector<int32_t> col2 = {1, 3, 0};
        CHECK(!undirected(3, ptr2.data(), col2.data(), g));
        std::vector<int64_t> ptr3 = {1, 1, 2, 3};
        CHECK(!undirected(3, ptr3.data(), col.data(), g));
    }
    if (failures) {
        printf("%d checks failed\n", failures);
        return 1;
    }
    printf("partition: all checks passed\n");
    return 0;
}
