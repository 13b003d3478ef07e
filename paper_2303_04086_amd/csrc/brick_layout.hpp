// Storage order of a level's two cubes on the device: the hash table H
// (side mbar) and the offset table Phi (side rbar) of Sec. 4.1.  Cells are
// grouped into bricks of 8 x 4 x 1 cells (32 entries, one 128-byte line of
// 4-byte entries), x fastest inside a brick and across bricks, over each z
// plane padded to whole bricks.  The eight corners of a cell then span 2.8
// lines on average instead of 4.1.  The index of cell (x, y, z) is the sum
// of one term per axis, so the index of a cell's corners is two additions of
// terms computed once per axis value.
// Shared by the host placement (psh.cpp) and the device lookups.
#pragma once

#include <stdint.h>

namespace inrf {

constexpr int kBrickX = 8, kBrickY = 4, kBrickZ = 1;
static_assert(kBrickX * kBrickY * kBrickZ == 32, "a brick is one 128-byte line of 4-byte entries");
static_assert(kBrickZ == 1, "the z term below assumes one plane per brick");

#if defined(__HIPCC__)
#define INRF_HD __host__ __device__
#else
#define INRF_HD
#endif

INRF_HD inline uint32_t brick_umul(uint32_t a, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul24(a, b);  // both factors below 2^24 for sides <= 1024
#else
    return a * b;
#endif
}

// Bricks along x, and the entry strides of one brick row and one brick plane.
INRF_HD inline uint32_t bricks_x(int side) { return uint32_t(side + kBrickX - 1) / kBrickX; }
INRF_HD inline uint32_t brick_row(int side) { return 32u * bricks_x(side); }
INRF_HD inline uint32_t brick_plane(int side) { return brick_row(side) * (uint32_t(side + kBrickY - 1) / kBrickY); }
// Entries a cube of the given side occupies.
INRF_HD inline int64_t brick_entries(int side) { return int64_t(brick_plane(side)) * side; }

// Per-axis terms, written as the linear part plus a correction per brick
// step so that each is a shift and a multiply-add:
//   x: (x / 8) * 32 + x % 8            = x + 24 (x / 8)
//   y: (y / 4) * row + 8 (y % 4)       = 8 y + (row - 32) (y / 4)
//   z: z * plane
INRF_HD inline uint32_t brick_x(uint32_t x) { return x + brick_umul(32u - kBrickX, x / kBrickX); }
INRF_HD inline uint32_t brick_y(uint32_t y, uint32_t row) {
    return kBrickX * y + brick_umul(row - 32u, y / kBrickY);
}
INRF_HD inline uint32_t brick_z(uint32_t z, uint32_t plane) { return brick_umul(z, plane); }

#undef INRF_HD

}  // namespace inrf
