// schedule.hpp -- wave schedules of the tiled coordinate-descent sweeps.
// Plain host C++ (no HIP), so the schedules can be tested on their own.
//
// A sweep is a list of waves; the tiles of one wave run concurrently, so the
// rows of the maintained product they update must be disjoint: a Theta tile
// (I, J) updates V[I, :] and reads Sigma[J, :] (waves row- and
// column-disjoint), a Lambda tile (I, J) updates U[I, :] and U[J, :] (the
// index blocks of a wave pairwise disjoint).
#pragma once

#include <stdint.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "tile_rect.hpp"

namespace cggm {

// Wave schedules of the coordinate-descent sweeps (host lists of rects with
// offsets of each wave; uploaded once per solve).
struct Schedule {
    std::vector<TileRect> rects;
    std::vector<int> wave_start;   // wave w = rects[wave_start[w], wave_start[w+1])
    int max_wave = 0;
    int waves() const { return (int)wave_start.size() - 1; }
    void finish_wave() {
        const int prev = wave_start.empty() ? 0 : wave_start.back();
        max_wave = std::max(max_wave, (int)rects.size() - prev);
        wave_start.push_back((int)rects.size());
    }
};

inline TileRect rect(int64_t r0, int64_t r1, int64_t c0, int64_t c1) {
    return TileRect{(int32_t)r0, (int32_t)r1, (int32_t)c0, (int32_t)c1};
}

// Theta: tile (I, J) belongs to wave (J - I) mod W, W = max(#row blocks,
// #column blocks); each wave is row- and column-disjoint.
inline Schedule theta_schedule(int64_t p, int64_t q, int tile, bool sequential) {
    Schedule s;
    s.wave_start.push_back(0);
    if (sequential) {
        for (int64_t i = 0; i < p; ++i)
            for (int64_t j = 0; j < q; ++j) {
                s.rects.push_back(rect(i, i + 1, j, j + 1));
                s.finish_wave();
            }
        return s;
    }
    const int64_t P = (p + tile - 1) / tile, Q = (q + tile - 1) / tile, W = std::max(P, Q);
    for (int64_t w = 0; w < W; ++w) {
        for (int64_t I = 0; I < P; ++I) {
            const int64_t J = (I + w) % W;
            if (J >= Q) continue;
            s.rects.push_back(rect(I * tile, std::min(p, (I + 1) * tile), J * tile,
                                   std::min(q, (J + 1) * tile)));
        }
        s.finish_wave();
    }
    return s;
}

// Theta by row groups (block-wise mode): the row tiles are taken in groups of
// `group` consecutive row tiles, and each group's tiles are scheduled like the
// whole matrix above -- tile (I, J) of the group in wave (J - I') mod W_g,
// I' = I - first row tile of the group, W_g = max(#row tiles of the group,
// #column blocks) -- so every wave is row- and column-disjoint and lies in one
// group, and the waves of a group are consecutive (the group's Sxx columns
// are formed once per sweep).  With group >= #row tiles it is theta_schedule.
inline Schedule theta_schedule_grouped(int64_t p, int64_t q, int tile, int64_t group) {
    Schedule s;
    s.wave_start.push_back(0);
    const int64_t P = (p + tile - 1) / tile, Q = (q + tile - 1) / tile;
    for (int64_t g0 = 0; g0 < P; g0 += group) {
        const int64_t G = std::min(group, P - g0), W = std::max(G, Q);
        for (int64_t w = 0; w < W; ++w) {
            bool any = false;
            for (int64_t I = 0; I < G; ++I) {
                const int64_t J = (I + w) % W;
                if (J >= Q) continue;
                const int64_t r = g0 + I;
                s.rects.push_back(rect(r * tile, std::min(p, (r + 1) * tile), J * tile,
                                       std::min(q, (J + 1) * tile)));
                any = true;
            }
            if (any) s.finish_wave();
        }
    }
    return s;
}

// Lambda: first the wave of all diagonal tiles, then the rounds of a
// round-robin pairing of the column blocks (each block once per round).
inline Schedule lambda_schedule(int64_t q, int tile, bool sequential) {
    Schedule s;
    s.wave_start.push_back(0);
    if (sequential) {
        for (int64_t i = 0; i < q; ++i)
            for (int64_t j = i; j < q; ++j) {
                s.rects.push_back(rect(i, i + 1, j, j + 1));
                s.finish_wave();
            }
        return s;
    }
    const int64_t Q = (q + tile - 1) / tile;
    auto blk = [&](int64_t I, int64_t J) {
        return rect(I * tile, std::min(q, (I + 1) * tile), J * tile, std::min(q, (J + 1) * tile));
    };
    for (int64_t I = 0; I < Q; ++I) s.rects.push_back(blk(I, I));
    s.finish_wave();
    const int64_t n = Q + (Q & 1);             // even number of slots (one bye if Q odd)
    for (int64_t r = 0; r + 1 < n; ++r) {
        std::vector<std::pair<int64_t, int64_t>> pairs;
        pairs.push_back({r, n - 1});
        for (int64_t k = 1; k < n / 2; ++k)
            pairs.push_back({(r + k) % (n - 1), (r - k + (n - 1)) % (n - 1)});
        bool any = false;
        for (auto [a, b] : pairs) {
            if (a >= Q || b >= Q) continue;     // bye
            const int64_t I = std::min(a, b), J = std::max(a, b);
            s.rects.push_back(blk(I, J));
            any = true;
        }
        if (any) s.finish_wave();
    }
    return s;
}

// The schedule with every wave split into min(parts, wave size) consecutive
// sub-waves of near-equal size: the same rects in the same order (so the
// device copy of the rects serves both), fewer tiles running concurrently.
inline Schedule split_waves(const Schedule &src, int parts) {
    Schedule s;
    s.rects = src.rects;
    s.wave_start.push_back(0);
    for (int w = 0; w < src.waves(); ++w) {
        const int b = src.wave_start[w], m = src.wave_start[w + 1] - b;
        const int k = std::max(1, std::min(parts, m));
        for (int i = 1; i <= k; ++i) {
            const int end = b + (int)((int64_t)m * i / k);
            if (end > s.wave_start.back()) {
                s.max_wave = std::max(s.max_wave, end - s.wave_start.back());
                s.wave_start.push_back(end);
            }
        }
    }
    return s;
}

}  // namespace cggm
