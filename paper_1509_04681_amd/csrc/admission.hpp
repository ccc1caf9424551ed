// admission.hpp -- device-pool bookkeeping and the admission rule of the
// request server.  Plain host C++ (no HIP), so the rule can be tested on its own.
#pragma once

#include <stddef.h>

#include <deque>
#include <iterator>
#include <map>

namespace cggm {

// First-fit allocator over one block of `size` bytes (offsets only; the
// memory itself belongs to the caller).  Free blocks are kept by offset and
// merged with their neighbours when a block is given back.
struct Pool {
    size_t size = 0;
    std::map<size_t, size_t> free_;   // offset -> bytes

    void init(size_t bytes) {
        size = bytes;
        free_.clear();
        if (bytes) free_[0] = bytes;
    }
    bool take(size_t bytes, size_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t o = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[o + bytes] = rest;
            *off = o;
            return true;
        }
        return false;
    }
    void give(size_t off, size_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t free_bytes() const {
        size_t b = 0;
        for (const auto &kv : free_) b += kv.second;
        return b;
    }
};

// The next queued item to start, removed from the queue with its block
// reserved (item->offset); nullptr if none can start now.  The head goes
// first; a later item whose footprint fits may pass a head that does not, at
// most max_bypass times in a row for the same head (head_bypassed counts them
// and is reset when the head starts).  Item needs `footprint` and `offset`.
template <class Item>
Item *admit_next(std::deque<Item *> &queue, Pool &pool, int &head_bypassed, int max_bypass) {
    if (queue.empty()) return nullptr;
    size_t off = 0;
    Item *h = queue.front();
    if (pool.take(h->footprint, &off)) {
        h->offset = off;
        queue.pop_front();
        head_bypassed = 0;
        return h;
    }
    if (head_bypassed >= max_bypass) return nullptr;
    for (auto it = std::next(queue.begin()); it != queue.end(); ++it) {
        if (pool.take((*it)->footprint, &off)) {
            Item *j = *it;
            j->offset = off;
            queue.erase(it);
            ++head_bypassed;
            return j;
        }
    }
    return nullptr;
}

}  // namespace cggm
