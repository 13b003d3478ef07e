// Memory images of the proxy BVH, shared by the host builder and the
// traversal kernels.
//
// Node (128 bytes, four children): the children's boxes as structure of
// arrays (min x of children 0..3, min y, min z, max x, max y, max z), then
// four child references.  A reference >= 0 is a node index; a negative
// reference r encodes a leaf, ~r = first << 3 | count (1..4 triangles starting
// at `first` in the triangle image); -1 marks an unused slot.  Node 0 is the
// root.  Boxes are the exact FP32 min/max of the triangles below.  The image
// is built as a binary SAH hierarchy and then collapsed to four-wide nodes,
// which halves the dependent node fetches of a traversal.
//
// Triangle (48 bytes, leaf order): v0.xyz + original index (as int bits),
// v1.xyz + 0, v2.xyz + 0.
#pragma once

#include <cstdint>

namespace inrf {

struct alignas(16) BvhNode {
    float lox[4], loy[4], loz[4];
    float hix[4], hiy[4], hiz[4];
    int32_t child[4];
    int32_t pad[4];
};
static_assert(sizeof(BvhNode) == 128, "node image is 128 bytes");

constexpr int32_t kBvhEmpty = -1;

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
constexpr int kBvhMaxDepth = 32;   // binary hierarchy before collapsing
constexpr int kBvhMaxStack = 64;   // traversal stack entries a hierarchy may need

inline int32_t bvh_leaf_ref(int32_t first, int32_t count) { return ~((first << 3) | count); }

}  // namespace inrf
