// Memory images of the proxy BVH, shared by the host builder and the
// traversal kernels.
//
// Node (64 bytes, one per interior split): the boxes of both children, so a
// visit tests two boxes with one 64-byte read.  A child reference >= 0 is a
// node index; a negative reference r encodes a leaf, ~r = first << 3 | count
// (count 0..4 triangles starting at `first` in the triangle image).  Node 0 is
// the root; a proxy of <= 4 triangles is a root with one leaf and one empty
// leaf.  Boxes are the exact FP32 min/max of the triangles below.
//
// Triangle (48 bytes, leaf order): v0.xyz + original index (as int bits),
// v1.xyz + 0, v2.xyz + 0.
#pragma once

#include <cstdint>

namespace inrf {

struct alignas(16) BvhNode {
    float lmin[3];
    float lmax[3];
    float rmin[3];
    float rmax[3];
    int32_t left, right;
    int32_t pad[2];
};
static_assert(sizeof(BvhNode) == 64, "node image is 64 bytes");

struct alignas(16) BvhTri {
    float v0[3];
    int32_t index;
    float v1[3];
    int32_t pad1;
    float v2[3];
    int32_t pad2;
};
static_assert(sizeof(BvhTri) == 48, "triangle image is 48 bytes");

constexpr int kBvhMaxLeaf = 4;
constexpr int kBvhMaxDepth = 32;

inline int32_t bvh_leaf_ref(int32_t first, int32_t count) { return ~((first << 3) | count); }

}  // namespace inrf
