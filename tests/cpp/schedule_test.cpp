// Host test of the coordinate-descent wave schedules (schedule.hpp): every
// tile exactly once, the tiles of a wave write disjoint rows of the
// maintained product, rects inside the matrix, ragged edges exact.
#include <stdio.h>
#include <stdlib.h>

#include <map>
#include <set>
#include <string>
#include <utility>

#include "schedule.hpp"

using namespace cggm;

static int checks = 0;
#define CHECK(c)                                                           \
    do {                                                                   \
        ++checks;                                                          \
        if (!(c)) {                                                        \
            fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #c); \
            exit(1);                                                       \
        }                                                                  \
    } while (0)

static void check_waves(const Schedule &s) {
    CHECK(!s.wave_start.empty() && s.wave_start.front() == 0);
    CHECK(s.wave_start.back() == (int)s.rects.size());
    int mx = 0;
    for (int w = 0; w < s.waves(); ++w) {
        CHECK(s.wave_start[w + 1] > s.wave_start[w]);          // no empty wave
        mx = std::max(mx, s.wave_start[w + 1] - s.wave_start[w]);
    }
    CHECK(mx == s.max_wave);
}

static void theta(int64_t p, int64_t q, int tile) {
    const Schedule s = theta_schedule(p, q, tile, false);
    check_waves(s);
    std::set<std::pair<int, int>> seen;
    int64_t cells = 0;
    for (int w = 0; w < s.waves(); ++w) {
        std::set<int> rows, cols;
        for (int k = s.wave_start[w]; k < s.wave_start[w + 1]; ++k) {
            const TileRect &r = s.rects[k];
            CHECK(0 <= r.r0 && r.r0 < r.r1 && r.r1 <= p && 0 <= r.c0 && r.c0 < r.c1 && r.c1 <= q);
            CHECK(r.r0 % tile == 0 && r.c0 % tile == 0);
            CHECK(r.r1 - r.r0 == std::min<int64_t>(tile, p - r.r0));
            CHECK(r.c1 - r.c0 == std::min<int64_t>(tile, q - r.c0));
            CHECK(rows.insert(r.r0).second);                    // row-disjoint (V rows)
            CHECK(cols.insert(r.c0).second);                    // column-disjoint
            CHECK(seen.insert({r.r0, r.c0}).second);            // each tile once
            cells += (int64_t)(r.r1 - r.r0) * (r.c1 - r.c0);
        }
    }
    CHECK(cells == p * q);
}

static void lambda(int64_t q, int tile) {
    const Schedule s = lambda_schedule(q, tile, false);
    check_waves(s);
    const int64_t Q = (q + tile - 1) / tile;
    std::set<std::pair<int, int>> seen;
    int64_t cells = 0;
    for (int w = 0; w < s.waves(); ++w) {
        std::set<int> blocks;
        for (int k = s.wave_start[w]; k < s.wave_start[w + 1]; ++k) {
            const TileRect &r = s.rects[k];
            CHECK(0 <= r.r0 && r.r0 < r.r1 && r.r1 <= q && 0 <= r.c0 && r.c0 < r.c1 && r.c1 <= q);
            CHECK(r.r0 <= r.c0);                                // upper triangle
            CHECK(seen.insert({r.r0, r.c0}).second);            // each tile once
            // U rows of both index blocks are written: pairwise disjoint blocks
            CHECK(blocks.insert(r.r0).second);
            if (r.c0 != r.r0) CHECK(blocks.insert(r.c0).second);
            cells += (int64_t)(r.r1 - r.r0) * (r.c1 - r.c0);
        }
        if (w == 0)                                             // the diagonal wave first
            for (int k = s.wave_start[0]; k < s.wave_start[1]; ++k)
                CHECK(s.rects[k].r0 == s.rects[k].c0);
    }
    CHECK((int64_t)seen.size() == Q * (Q + 1) / 2);
    // blocks of the upper triangle including the diagonal ones, in cells
    int64_t expect = 0;
    for (int64_t I = 0; I < Q; ++I)
        for (int64_t J = I; J < Q; ++J)
            expect += (std::min<int64_t>(q, (I + 1) * tile) - I * tile) *
                      (std::min<int64_t>(q, (J + 1) * tile) - J * tile);
    CHECK(cells == expect);
    // the round-robin pairing needs Q - 1 rounds (Q even) or Q (Q odd)
    CHECK(s.waves() == 1 + (Q > 1 ? (Q % 2 == 0 ? Q - 1 : Q) : 0));
}

static void sequential(int64_t p, int64_t q) {
    const Schedule t = theta_schedule(p, q, 64, true);
    CHECK(t.waves() == p * q && t.max_wave == 1);
    for (int64_t k = 0; k < p * q; ++k)                         // row-major order
        CHECK(t.rects[k].r0 == k / q && t.rects[k].c0 == k % q &&
              t.rects[k].r1 == t.rects[k].r0 + 1 && t.rects[k].c1 == t.rects[k].c0 + 1);
    const Schedule l = lambda_schedule(q, 64, true);
    CHECK(l.waves() == q * (q + 1) / 2 && l.max_wave == 1);
    int k = 0;
    for (int64_t i = 0; i < q; ++i)                             // lexicographic, i <= j
        for (int64_t j = i; j < q; ++j, ++k) CHECK(l.rects[k].r0 == i && l.rects[k].c0 == j);
}

static void split(int64_t q, int parts) {
    const Schedule s = lambda_schedule(q, 64, false);
    const Schedule t = split_waves(s, parts);
    check_waves(t);
    CHECK(t.rects.size() == s.rects.size());
    for (size_t k = 0; k < s.rects.size(); ++k)                 // same rects, same order
        CHECK(t.rects[k].r0 == s.rects[k].r0 && t.rects[k].c0 == s.rects[k].c0);
    // every original wave boundary is kept and each wave becomes
    // min(parts, size) sub-waves of near-equal size
    std::set<int> starts(t.wave_start.begin(), t.wave_start.end());
    int expect = 0;
    for (int w = 0; w < s.waves(); ++w) {
        CHECK(starts.count(s.wave_start[w]) && starts.count(s.wave_start[w + 1]));
        const int m = s.wave_start[w + 1] - s.wave_start[w];
        expect += std::min(parts, m);
        int lo = m, hi = 0, cnt = 0;
        for (int x = 0; x < t.waves(); ++x)
            if (t.wave_start[x] >= s.wave_start[w] && t.wave_start[x + 1] <= s.wave_start[w + 1]) {
                const int sz = t.wave_start[x + 1] - t.wave_start[x];
                lo = std::min(lo, sz), hi = std::max(hi, sz), ++cnt;
            }
        CHECK(cnt == std::min(parts, m) && hi - lo <= 1);
    }
    CHECK(t.waves() == expect);
    if (parts == 1) CHECK(t.wave_start == s.wave_start);
}

// "dump q tile parts": print the Lambda schedule of a q x q problem with the
// given tile edge, every wave split into `parts` sub-waves, one sub-wave per
// line as "r0 r1 c0 c1" groups (read by the CPU emulation of the tiled
// direction in tests/test_split_emulation_cpu.py).
static int dump(int64_t q, int tile, int parts) {
    const Schedule s = split_waves(lambda_schedule(q, tile, false), parts);
    for (int w = 0; w < s.waves(); ++w) {
        for (int k = s.wave_start[w]; k < s.wave_start[w + 1]; ++k)
            printf("%s%d %d %d %d", k > s.wave_start[w] ? " " : "", s.rects[k].r0,
                   s.rects[k].r1, s.rects[k].c0, s.rects[k].c1);
        printf("\n");
    }
    return 0;
}

// Grouped Theta schedule: every tile once, waves row- and column-disjoint,
// each wave inside one group of `group` row tiles, the waves of a group
// consecutive; with one group it equals theta_schedule.
static void theta_grouped(int64_t p, int64_t q, int tile, int64_t group) {
    const Schedule s = theta_schedule_grouped(p, q, tile, group);
    check_waves(s);
    const int64_t P = (p + tile - 1) / tile, Q = (q + tile - 1) / tile;
    std::set<std::pair<int, int>> seen;
    int64_t last_group = -1;
    for (int w = 0; w < s.waves(); ++w) {
        std::set<int> rows, cols;
        const int64_t g = (s.rects[s.wave_start[w]].r0 / tile) / group;
        CHECK(g >= last_group);                       // groups in order, consecutive
        last_group = g;
        for (int k = s.wave_start[w]; k < s.wave_start[w + 1]; ++k) {
            const TileRect &r = s.rects[k];
            CHECK((r.r0 / tile) / group == g);
            CHECK(rows.insert(r.r0).second && cols.insert(r.c0).second);
            CHECK(r.r0 % tile == 0 && r.c0 % tile == 0);
            CHECK(r.r1 == std::min<int64_t>(p, r.r0 + tile));
            CHECK(r.c1 == std::min<int64_t>(q, r.c0 + tile));
            CHECK(seen.insert({r.r0, r.c0}).second);
        }
    }
    CHECK((int64_t)seen.size() == P * Q);
    if (group >= P) {
        const Schedule t = theta_schedule(p, q, tile, false);
        CHECK(t.wave_start == s.wave_start);
        for (size_t k = 0; k < t.rects.size(); ++k)
            CHECK(t.rects[k].r0 == s.rects[k].r0 && t.rects[k].c0 == s.rects[k].c0);
    }
}

int main(int argc, char **argv) {
    if (argc == 5 && std::string(argv[1]) == "dump")
        return dump(atoll(argv[2]), atoi(argv[3]), atoi(argv[4]));
    const int64_t sizes[] = {1, 2, 63, 64, 65, 127, 128, 130, 515, 640, 1000};
    for (int64_t p : sizes)
        for (int64_t q : sizes) theta(p, q, 64);
    theta(20000, 20000, 64);
    theta(530, 515, 32);
    for (int64_t q : sizes) lambda(q, 64);
    for (int64_t q : {64 * 7, 64 * 8 + 5, 20000}) lambda(q, 64);
    lambda(515, 32);
    for (int parts : {1, 2, 3, 4, 64, 1000})
        for (int64_t q : {64, 130, 640, 1000, 20000}) split(q, parts);
    for (int64_t group : {1, 2, 3, 5, 64, 1000})
        for (int64_t p : {1, 64, 130, 700, 2000})
            for (int64_t q : {1, 65, 640}) theta_grouped(p, q, 64, group);
    theta_grouped(20000, 4000, 64, 83);
    sequential(5, 7);
    sequential(1, 1);
    printf("schedule: %d checks passed\n", checks);
    return 0;
}
