// tile_rect.hpp -- a rectangle of coordinates of a coordinate-descent tile.
#pragma once

#include <stdint.h>

namespace cggm {

struct TileRect {
    int32_t r0, r1, c0, c1;   // rows [r0, r1), columns [c0, c1)
};

}  // namespace cggm
