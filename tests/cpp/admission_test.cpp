// Host test of the request server's pool and admission rule (admission.hpp).
// Prints one line per check and exits non-zero on the first failure.
#include <stdio.h>
#include <stdlib.h>

#include <deque>
#include <random>
#include <vector>

#include "admission.hpp"

using cggm::Pool;
using cggm::admit_next;

struct Item {
    size_t footprint = 0, offset = 0;
    int id = 0;
};

static int checks = 0;
#define CHECK(c)                                                           \
    do {                                                                   \
        ++checks;                                                          \
        if (!(c)) {                                                        \
            fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #c); \
            exit(1);                                                       \
        }                                                                  \
    } while (0)

static void test_first_fit_and_merge() {
    Pool p;
    p.init(1000);
    size_t a, b, c, d;
    CHECK(p.take(300, &a) && a == 0);
    CHECK(p.take(300, &b) && b == 300);
    CHECK(p.take(300, &c) && c == 600);
    CHECK(!p.take(200, &d));               // 100 left
    p.give(b, 300);                        // hole in the middle
    CHECK(p.take(200, &d) && d == 300);    // first fit takes the hole
    p.give(d, 200);
    p.give(a, 300);                        // merges with [300, 600)
    CHECK(p.free_.size() == 2 && p.free_.begin()->second == 600);
    p.give(c, 300);                        // everything merges back into one block
    CHECK(p.free_.size() == 1 && p.free_.begin()->first == 0 &&
          p.free_.begin()->second == 1000);
}

static void test_random_take_give_conserves() {
    std::mt19937_64 rng(7);
    Pool p;
    p.init(1 << 20);
    struct Blk { size_t off, bytes; };
    std::vector<Blk> held;
    for (int it = 0; it < 20000; ++it) {
        if (!held.empty() && (rng() % 2)) {
            const size_t k = rng() % held.size();
            p.give(held[k].off, held[k].bytes);
            held.erase(held.begin() + k);
        } else {
            const size_t bytes = 1 + rng() % 50000;
            size_t off;
            if (p.take(bytes, &off)) {
                for (const Blk &h : held)        // no overlap with held blocks
                    CHECK(off + bytes <= h.off || h.off + h.bytes <= off);
                CHECK(off + bytes <= p.size);
                held.push_back({off, bytes});
            }
        }
        size_t used = 0;
        for (const Blk &h : held) used += h.bytes;
        CHECK(used + p.free_bytes() == p.size);
    }
    for (const Blk &h : held) p.give(h.off, h.bytes);
    CHECK(p.free_.size() == 1 && p.free_.begin()->second == p.size);
}

static void test_admission_order_and_bypass() {
    Pool p;
    p.init(100);
    std::vector<Item> items(6);
    const size_t fp[6] = {60, 50, 30, 20, 10, 100};
    for (int k = 0; k < 6; ++k) items[k] = {fp[k], 0, k};
    std::deque<Item *> q;
    for (auto &it : items) q.push_back(&it);
    int bypassed = 0;
    Item *a = admit_next(q, p, bypassed, 2);
    CHECK(a && a->id == 0);                  // head first
    Item *b = admit_next(q, p, bypassed, 2);
    CHECK(b && b->id == 2 && bypassed == 1); // 50 does not fit in 40: 30 passes it
    Item *c = admit_next(q, p, bypassed, 2);
    CHECK(c && c->id == 4 && bypassed == 2); // 20 does not fit in 10 either: 10 passes
    Item *d = admit_next(q, p, bypassed, 2);
    CHECK(!d);                               // bypass limit for this head reached
    p.give(a->offset, a->footprint);         // 60 back: the head (50) fits now
    Item *e = admit_next(q, p, bypassed, 2);
    CHECK(e && e->id == 1 && bypassed == 0);
    CHECK(!admit_next(q, p, bypassed, 2));   // the new head (20) does not fit in the 10 left
    p.give(b->offset, b->footprint);
    p.give(c->offset, c->footprint);
    p.give(e->offset, e->footprint);
    while (!q.empty()) {                     // with everything free the rest drains in order
        Item *g = admit_next(q, p, bypassed, 2);
        CHECK(g);
        p.give(g->offset, g->footprint);
    }
    CHECK(p.free_bytes() == 100);
}

static void test_no_bypass_is_fifo() {
    Pool p;
    p.init(100);
    std::vector<Item> items = {{90, 0, 0}, {20, 0, 1}, {5, 0, 2}};
    std::deque<Item *> q = {&items[0], &items[1], &items[2]};
    int bypassed = 0;
    Item *a = admit_next(q, p, bypassed, 0);
    CHECK(a && a->id == 0);
    CHECK(!admit_next(q, p, bypassed, 0));   // 20 waits, and 5 may not pass it
    p.give(a->offset, a->footprint);
    Item *b = admit_next(q, p, bypassed, 0);
    Item *c = admit_next(q, p, bypassed, 0);
    CHECK(b && c && b->id == 1 && c->id == 2);
}

int main() {
    test_first_fit_and_merge();
    test_random_take_give_conserves();
    test_admission_order_and_bypass();
    test_no_bypass_is_fifo();
    printf("admission: %d checks passed\n", checks);
    return 0;
}
