// Scenes of several objects (each an i-NOLF in its own unit cube, placed by a
// similarity transform), merged per ray by depth as the paper's frame
// composer merges objects (Sec. 5).  Included by render.hip after the trace
// kernels, whose ray generation, packet traversal and record layout it
// reuses.
//
// k_trace_scene: per camera wave, the objects are visited in index order;
// an object is skipped unless some lane's ray meets its world box before the
// lane's current closest hit.  A visited object's BVH is traversed as one
// packet with the ray mapped to object space (the ray parameter t is the same
// in both spaces, so hits compare directly); a later object replaces a hit
// only if strictly nearer, so equal t goes to the lower index.  Hit records
// hold the object-space hit point and unit direction and the object index,
// and are written per tile grouped by object; the scan and compaction then
// give one contiguous run of records per object, which the shading kernel
// of that object processes.
#pragma once

namespace inrf {
namespace dev {

constexpr int kMaxObjects = INRF_MAX_OBJECTS;

struct ObjC {
    float m[9];                 // world -> object, linear part R^T / s (row-major)
    float c[3];                 // world -> object, offset -R^T t / s
    float lo[3], hi[3];         // world bounds of the object's unit cube
    const BvhNode* nodes;
    const BvhTri* tris;
    int32_t n_tris, stack_depth;
};

struct SceneC {
    int32_t n_objs, pad;
    ObjC o[kMaxObjects];
};

struct SceneArgs {
    float* rgba;     // zero colour of misses
    float* depth;    // nullable
    int32_t* tri;    // nullable
    int32_t* obj;    // nullable
    HitRec* tmp;     // hit records of tile b at blk[k * n_tiles + b].y, object k
    int2* blk;       // [n_objs][n_tiles]: (hits of object k in tile b, first record in tmp)
};

__device__ __forceinline__ float3 xform(const float* m, const float* c, float3 v, bool point) {
    float3 r = make_float3(m[0] * v.x + m[1] * v.y + m[2] * v.z, m[3] * v.x + m[4] * v.y + m[5] * v.z,
                           m[6] * v.x + m[7] * v.y + m[8] * v.z);
    if (point) r = make_float3(r.x + c[0], r.y + c[1], r.z + c[2]);
    return r;
}

// One workgroup per 16x16 tile of the cameras of `cams` (camera j owns
// tiles [c[j].tile0, c[j+1].tile0) and pixels from c[j].pix0 on), so the
// rays of several requests are traced by one launch and their records are
// grouped by object across all of them.
template <int NCAM>
__global__ __launch_bounds__(kThreads) void k_trace_scene(SceneC sc, CamSet<NCAM> cams, SceneArgs a, int n_tiles) {
    __shared__ int wst[(kThreads / 64) * kBvhMaxStack];
    __shared__ int s_cnt[kThreads / 64][kMaxObjects];
    const int lane = __lane_id(), wave = int(threadIdx.x) / 64;
    const int b = blockIdx.x;
    int j = 0;  // the camera of this tile (wave-uniform)
    for (int k = 1; k < NCAM && k < cams.n; ++k)
        if (b >= cams.c[k].tile0) j = k;
    const CamC& cam = cams.c[j];
    int tx, ty;
    tile_at(b - cam.tile0, cam.tiles_x, (cam.H + kTile - 1) / kTile, tx, ty);
    const int row = ty * kTile + 8 * (wave >> 1) + (lane >> 3), col = tx * kTile + 8 * (wave & 1) + (lane & 7);
    const bool valid = row < cam.H && col < cam.W;
    const int64_t ray = cam.pix0 + int64_t(row) * cam.W + col;
    const int64_t base =
        cam.pix0 + int64_t(ty) * kTile * cam.W + int64_t(tx) * kTile * min(kTile, cam.H - ty * kTile);
    const float3 d = camera_dir(cam, row, col);
    const float3 o = make_float3(cam.o[0], cam.o[1], cam.o[2]);
    const RayPre Rw = ray_setup(o, d);

    float best_t = INFINITY;
    int32_t best_i = -1, best_k = -1;
    for (int k = 0; k < sc.n_objs; ++k) {
        const ObjC& ob = sc.o[k];
        float tn;
        const bool in_box = valid && hit_box(Rw, ob.lo[0], ob.lo[1], ob.lo[2], ob.hi[0], ob.hi[1], ob.hi[2], best_t, tn);
        if (__ballot(in_box) == 0) continue;
        const float3 oo = xform(ob.m, ob.c, o, true), dd = xform(ob.m, ob.c, d, false);
        const RayPre Ro = ray_setup(oo, dd);
        float t_k = best_t;
        int32_t i_k = -1;  // an equal t cannot replace the earlier object
        closest_hit_packet(ob, Ro, in_box, wst + wave * kBvhMaxStack, t_k, i_k);
        if (i_k >= 0) {
            best_t = t_k;
            best_i = i_k;
            best_k = k;
        }
    }
    const bool hit = best_k >= 0;
    if (valid) {
        if (a.depth) a.depth[ray] = best_t;
        if (a.tri) a.tri[ray] = best_i;
        if (a.obj) a.obj[ray] = best_k;
        if (!hit) reinterpret_cast<float4*>(a.rgba)[ray] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    // per-object counts of the tile, then records grouped by object
    int my_before = 0;  // records of lower objects in this tile, plus those of lower waves for my object
    uint64_t my_mask = 0;
    for (int k = 0; k < sc.n_objs; ++k) {
        const uint64_t mk = __ballot(hit && best_k == k);
        if (lane == 0) s_cnt[wave][k] = __popcll(mk);
        if (best_k == k) my_mask = mk;
    }
    __syncthreads();
    int lower_objects = 0;
    for (int k = 0; k < sc.n_objs; ++k) {
        int tile_k = 0, waves_before = 0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) {
            tile_k += s_cnt[w][k];
            waves_before += w < wave ? s_cnt[w][k] : 0;
        }
        if (best_k == k) my_before = lower_objects + waves_before;
        if (threadIdx.x == 0) a.blk[int64_t(k) * n_tiles + b] = make_int2(tile_k, int(base) + lower_objects);
        lower_objects += tile_k;
    }
    if (hit) {
        const int64_t pos = base + my_before + __popcll(my_mask & ((uint64_t(1) << lane) - 1));
        HitRec h;
        for (int k = 0; k < sc.n_objs; ++k) {  // object-space point and direction of the winner
            if (best_k != k) continue;
            const ObjC& ob = sc.o[k];
            const float3 oo = xform(ob.m, ob.c, o, true), dd = xform(ob.m, ob.c, d, false);
            const float3 u = unit_of(dd);
            h.x = clamp01(oo.x + best_t * dd.x);
            h.y = clamp01(oo.y + best_t * dd.y);
            h.z = clamp01(oo.z + best_t * dd.z);
            h.dx = u.x;
            h.dy = u.y;
            h.dz = u.z;
        }
        h.out = int32_t(ray);
        h.pad = best_k;
        a.tmp[pos] = h;
    }
}

// First record of each object's run in the packed list: seg[k] is the packed
// offset of entry (k, tile 0); seg[n_objs] the total.
__global__ void k_segments(const int32_t* __restrict__ offsets, const int32_t* __restrict__ runs, int n_tiles,
                           int n_objs, const int32_t* __restrict__ counter, int32_t* __restrict__ seg) {
    const int k = threadIdx.x;
    if (k < n_objs) {
        const int e = k * n_tiles;
        seg[k] = offsets[e] + runs[e / kScanRun];
    } else if (k == n_objs) {
        seg[k] = *counter;
    }
}

}  // namespace dev
}  // namespace inrf
