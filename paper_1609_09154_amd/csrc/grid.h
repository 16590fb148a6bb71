// Launch-size cap shared by the kernels whose grids grow with the data.
#pragma once

#include <stdint.h>

namespace nmfk {

// A dispatch counts the work-items of each grid dimension in 32 bits, so a
// grid that grows with the data (rows x KP copies, one wavefront per row of a
// 10^8-row factor) is capped at GRID_CAP blocks and its kernel strides over
// the remaining blocks; below the cap the grid is unchanged.
constexpr int64_t GRID_CAP = (int64_t)1 << 20;
inline unsigned capped_grid(int64_t blocks) {
  return (unsigned)(blocks < 1 ? 1 : (blocks > GRID_CAP ? GRID_CAP : blocks));
}

}  // namespace nmfk
