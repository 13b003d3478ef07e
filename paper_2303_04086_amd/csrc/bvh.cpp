// Binned-SAH BVH over the proxy triangles (host) and the inrf_build_bvh*
// entry points.  The hierarchy only accelerates the closest-hit query; the
// result it must reach is the brute-force closest hit over all triangles.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "bvh_layout.hpp"
#include "host_common.hpp"

namespace inrf {
namespace {

struct Box {
    float lo[3] = {INFINITY, INFINITY, INFINITY};
    float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    void grow(const float* p) {
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], p[k]);
            hi[k] = std::max(hi[k], p[k]);
        }
    }
    void grow(const Box& b) {
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], b.lo[k]);
            hi[k] = std::max(hi[k], b.hi[k]);
        }
    }
    double area() const {
        if (lo[0] > hi[0]) return 0.0;
        const double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
        return 2.0 * (dx * dy + dy * dz + dz * dx);
    }
};

// Binary node during the build: both children's boxes and references
// (same reference encoding as the four-wide image).
struct BinNode {
    Box lb, rb;
    int32_t left, right;
};

struct Builder {
    const float* V;
    const int32_t* T;
    std::vector<Box> tb;         // triangle boxes
    std::vector<float> cen;      // centroids [n][3]
    std::vector<int32_t> order;  // triangle permutation
    std::vector<BinNode> nodes;
    int depth = 0;
    bool median_only = false;

    struct Range {
        int32_t b, e;
    };

    Box bounds(int32_t b, int32_t e) const {
        Box bx;
        for (int32_t i = b; i < e; ++i) bx.grow(tb[size_t(order[size_t(i)])]);
        return bx;
    }

    int32_t split(int32_t b, int32_t e) {
        const int32_t n = e - b;
        float clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int32_t i = b; i < e; ++i)
            for (int k = 0; k < 3; ++k) {
                const float c = cen[size_t(order[size_t(i)]) * 3 + k];
                clo[k] = std::min(clo[k], c);
                chi[k] = std::max(chi[k], c);
            }
        int axis = 0;
        for (int k = 1; k < 3; ++k)
            if (chi[k] - clo[k] > chi[axis] - clo[axis]) axis = k;
        auto median = [&] {
            const int32_t m = b + n / 2;
            std::nth_element(order.begin() + b, order.begin() + m, order.begin() + e, [&](int32_t x, int32_t y) {
                const float cx = cen[size_t(x) * 3 + axis], cy = cen[size_t(y) * 3 + axis];
                return cx < cy || (cx == cy && x < y);
            });
            return m;
        };
        if (median_only || !(chi[axis] > clo[axis])) return median();
        constexpr int NB = 32;
        double best = INFINITY;
        int best_axis = -1, best_bin = -1;
        for (int k = 0; k < 3; ++k) {
            if (!(chi[k] > clo[k])) continue;
            Box bb[NB];
            int cnt[NB] = {0};
            const double scale = NB / (double(chi[k]) - double(clo[k]));
            for (int32_t i = b; i < e; ++i) {
                const int32_t t = order[size_t(i)];
                int bin = int((double(cen[size_t(t) * 3 + k]) - clo[k]) * scale);
                bin = std::min(std::max(bin, 0), NB - 1);
                bb[bin].grow(tb[size_t(t)]);
                ++cnt[bin];
            }
            double right_area[NB];
            int right_cnt[NB];
            Box acc;
            int c = 0;
            for (int i = NB - 1; i > 0; --i) {
                acc.grow(bb[i]);
                c += cnt[i];
                right_area[i] = acc.area();
                right_cnt[i] = c;
            }
            Box lacc;
            int lc = 0;
            for (int i = 0; i < NB - 1; ++i) {
                lacc.grow(bb[i]);
                lc += cnt[i];
                if (lc == 0 || right_cnt[i + 1] == 0) continue;
                const double cost = lacc.area() * lc + right_area[i + 1] * right_cnt[i + 1];
                if (cost < best) {
                    best = cost;
                    best_axis = k;
                    best_bin = i;
                }
            }
        }
        if (best_axis < 0) return median();
        const double scale = NB / (double(chi[best_axis]) - double(clo[best_axis]));
        auto it = std::stable_partition(order.begin() + b, order.begin() + e, [&](int32_t t) {
            int bin = int((double(cen[size_t(t) * 3 + best_axis]) - clo[best_axis]) * scale);
            bin = std::min(std::max(bin, 0), NB - 1);
            return bin <= best_bin;
        });
        const int32_t m = int32_t(it - order.begin());
        return (m == b || m == e) ? median() : m;
    }

    // Returns the child reference for the range; builds nodes for interiors.
    int32_t build(int32_t b, int32_t e, int d) {
        depth = std::max(depth, d);
        if (e - b <= kBvhMaxLeaf) return bvh_leaf_ref(b, e - b);
        const int32_t id = int32_t(nodes.size());
        nodes.emplace_back();
        const int32_t m = split(b, e);
        const Box lb = bounds(b, m), rb = bounds(m, e);
        const int32_t l = build(b, m, d + 1);
        const int32_t r = build(m, e, d + 1);
        BinNode& nd = nodes[size_t(id)];
        nd.lb = lb;
        nd.rb = rb;
        nd.left = l;
        nd.right = r;
        return id;
    }

    void run(int64_t nt) {
        order.resize(size_t(nt));
        for (int64_t i = 0; i < nt; ++i) order[size_t(i)] = int32_t(i);
        nodes.clear();
        depth = 0;
        if (nt <= kBvhMaxLeaf) {
            BinNode root;
            root.lb = bounds(0, int32_t(nt));
            root.left = nt > 0 ? bvh_leaf_ref(0, int32_t(nt)) : kBvhEmpty;
            root.right = kBvhEmpty;
            nodes.push_back(root);
            depth = 2;
            return;
        }
        build(0, int32_t(nt), 1);  // depth = level of the deepest leaf, root = 1
    }
};

// Collapses the binary hierarchy into four-wide nodes: a node's slots start
// as its two children and the interior slot with the largest box area is
// replaced by its own two children until four slots are used or none is
// interior.  Also returns the traversal stack entries a ray can need: a node
// with k interior children defers up to k - 1 of them.
struct Collapser {
    const std::vector<BinNode>& bin;
    std::vector<BvhNode> out;
    int32_t depth = 0;

    struct Slot {
        int32_t ref;
        Box box;
    };

    // returns the stack need of the subtree rooted at the new node
    int32_t collapse(int32_t bin_id, int32_t level, int32_t* out_id) {
        depth = std::max(depth, level);
        Slot s[4];
        int n = 0;
        const BinNode& b = bin[size_t(bin_id)];
        if (b.left != kBvhEmpty) s[n++] = Slot{b.left, b.lb};
        if (b.right != kBvhEmpty) s[n++] = Slot{b.right, b.rb};
        while (n < 4) {
            int pick = -1;
            double best = -1.0;
            for (int i = 0; i < n; ++i)
                if (s[i].ref >= 0 && s[i].box.area() > best) {
                    best = s[i].box.area();
                    pick = i;
                }
            if (pick < 0) break;
            const BinNode& c = bin[size_t(s[pick].ref)];
            s[pick] = Slot{c.left, c.lb};
            if (c.right != kBvhEmpty) s[n++] = Slot{c.right, c.rb};
        }
        const int32_t id = int32_t(out.size());
        out.emplace_back();
        *out_id = id;
        int32_t child_ref[4] = {kBvhEmpty, kBvhEmpty, kBvhEmpty, kBvhEmpty};
        int interior = 0;
        int32_t sub = 0;
        for (int i = 0; i < n; ++i) {
            if (s[i].ref >= 0) {
                int32_t cid;
                sub = std::max(sub, collapse(s[i].ref, level + 1, &cid));
                child_ref[i] = cid;
                ++interior;
            } else {
                child_ref[i] = s[i].ref;
            }
        }
        BvhNode& nd = out[size_t(id)];
        for (int i = 0; i < 4; ++i) {
            const Box bx = i < n ? s[i].box : Box();
            nd.lox[i] = bx.lo[0];
            nd.loy[i] = bx.lo[1];
            nd.loz[i] = bx.lo[2];
            nd.hix[i] = bx.hi[0];
            nd.hiy[i] = bx.hi[1];
            nd.hiz[i] = bx.hi[2];
            nd.child[i] = child_ref[i];
            nd.pad[i] = 0;
        }
        return std::max(0, interior - 1) + sub;
    }
};

// Renumbers the nodes in breadth-first order (the root stays 0): the top
// levels of the hierarchy, which every ray visits, share cache lines and
// pages at the start of the image.
std::vector<BvhNode> breadth_first(const std::vector<BvhNode>& in) {
    std::vector<int32_t> order, renum(in.size(), -1);
    order.reserve(in.size());
    if (!in.empty()) order.push_back(0);
    for (size_t h = 0; h < order.size(); ++h) {
        renum[size_t(order[h])] = int32_t(h);
        for (int c = 0; c < 4; ++c) {
            const int32_t r = in[size_t(order[h])].child[c];
            if (r >= 0) order.push_back(r);
        }
    }
    std::vector<BvhNode> out(order.size());
    for (size_t h = 0; h < order.size(); ++h) {
        out[h] = in[size_t(order[h])];
        for (int c = 0; c < 4; ++c)
            if (out[h].child[c] >= 0) out[h].child[c] = renum[size_t(out[h].child[c])];
    }
    return out;
}

}  // namespace
}  // namespace inrf

struct inrf_bvh {
    std::vector<inrf::BvhNode> nodes;
    std::vector<inrf::BvhTri> tris;
    int32_t depth = 0;
    int32_t stack = 0;
};

using namespace inrf;

extern "C" {

inrf_status inrf_build_bvh(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris, inrf_bvh** out) {
    return guarded("inrf_build_bvh", [&] {
        require(out != nullptr, "out is NULL");
        *out = nullptr;
        require(n_verts >= 0 && n_tris >= 0, "negative sizes");
        require(n_tris < (int64_t(1) << 27), "too many triangles (limit 2^27)");
        require(n_verts == 0 || verts, "verts is NULL");
        require(n_tris == 0 || tris, "tris is NULL");
        for (int64_t i = 0; i < n_verts * 3; ++i) require(std::isfinite(verts[i]), "non-finite vertex");
        for (int64_t i = 0; i < n_tris * 3; ++i)
            require(tris[i] >= 0 && tris[i] < n_verts, "triangle vertex index out of range");
        Builder B{verts, tris, {}, {}, {}, {}, 0, false};
        B.tb.resize(size_t(n_tris));
        B.cen.resize(size_t(n_tris) * 3);
        for (int64_t t = 0; t < n_tris; ++t) {
            for (int v = 0; v < 3; ++v) B.tb[size_t(t)].grow(&verts[size_t(tris[t * 3 + v]) * 3]);
            for (int k = 0; k < 3; ++k) {
                double s = 0;
                for (int v = 0; v < 3; ++v) s += verts[size_t(tris[t * 3 + v]) * 3 + k];
                B.cen[size_t(t) * 3 + k] = float(s / 3.0);
            }
        }
        B.run(n_tris);
        if (B.depth > kBvhMaxDepth) {
            B.median_only = true;
            B.run(n_tris);
        }
        if (B.depth > kBvhMaxDepth) fail(INRF_E_BUILD, "hierarchy deeper than 32 levels");
        Collapser C{B.nodes, {}, 0};
        int32_t root = 0;
        const int32_t stack = C.collapse(0, 1, &root);
        if (stack > kBvhMaxStack) fail(INRF_E_BUILD, "traversal would need more than 64 stack entries");
        auto* obj = new inrf_bvh();
        obj->nodes = breadth_first(C.out);
        obj->depth = C.depth + 1;  // leaves sit below the deepest node
        obj->stack = std::max(1, stack);
        obj->tris.resize(size_t(n_tris));
        for (int64_t i = 0; i < n_tris; ++i) {
            const int32_t t = B.order[size_t(i)];
            BvhTri& d = obj->tris[size_t(i)];
            std::memset(&d, 0, sizeof(d));
            for (int k = 0; k < 3; ++k) {
                d.v0[k] = verts[size_t(tris[size_t(t) * 3 + 0]) * 3 + k];
                d.v1[k] = verts[size_t(tris[size_t(t) * 3 + 1]) * 3 + k];
                d.v2[k] = verts[size_t(tris[size_t(t) * 3 + 2]) * 3 + k];
            }
            d.index = t;
        }
        *out = obj;
    });
}

inrf_status inrf_bvh_get_info(const inrf_bvh* bvh, inrf_bvh_info* info) {
    return guarded("inrf_bvh_get_info", [&] {
        require(bvh && info, "NULL argument");
        info->n_nodes = int64_t(bvh->nodes.size());
        info->node_bytes = int64_t(bvh->nodes.size() * sizeof(BvhNode));
        info->tri_bytes = int64_t(bvh->tris.size() * sizeof(BvhTri));
        info->depth = bvh->depth;
        info->max_leaf = kBvhMaxLeaf;
        info->stack = bvh->stack;
        info->pad = 0;
    });
}

inrf_status inrf_bvh_copy(const inrf_bvh* bvh, void* nodes, void* tri_data) {
    return guarded("inrf_bvh_copy", [&] {
        require(bvh && nodes, "NULL argument");
        require(bvh->tris.empty() || tri_data, "tri_data is NULL");
        std::memcpy(nodes, bvh->nodes.data(), bvh->nodes.size() * sizeof(BvhNode));
        if (!bvh->tris.empty()) std::memcpy(tri_data, bvh->tris.data(), bvh->tris.size() * sizeof(BvhTri));
    });
}

void inrf_bvh_free(inrf_bvh* bvh) { delete bvh; }

}  // extern "C"
