// The paper's own i-NOLF hit estimator (Sec. 4.2): a march through cached
// density texture cubes.  The sample of largest blending weight is the hit
// point, the summed weights are the coarse opacity alpha_c fed to the
// network, and the diffuse texture cubes give the diffuse colour and the
// specular tint at the hit point, combined with the network's specular
// colour in the shading kernel (Eq. 6-7).  Included by render.hip after the
// trace kernels, whose tiling and hit-record layout it reuses.
//
// k_march: one camera ray per lane, 8x8 pixels per wave as in k_trace, each
// lane marching on its own.  Samples sit at t_in + (j + 1/2) step inside the
// unit cube.  A sample in an empty base cell jumps to the first sample at or
// after the cell's exit (less 1/100 of a step, so no sample of a following
// cell is ever skipped; empty cells hold zero density, so skipping their
// samples changes nothing).  The march ends after the first sample whose
// updated transmittance is below t_stop.  With power-of-two base and cube
// resolutions every cell, cube and weight computation from a position is
// exact in FP32.
#pragma once

namespace inrf {
namespace dev {

struct CubesC {
    const int32_t* index;  // [b^3] cube of each base cell, < 0: empty
    const __half* dens;    // [n_cubes][(r+1)^3]
    const __half* diff;    // [n_cubes][(r+1)^3][4]: diffuse RGB, tint
    int64_t n_cubes;
    int32_t b, r, r1;       // base and cube resolutions, r + 1
    int32_t j_max;          // bound on the samples of one ray (the cube's diagonal / step + 2)
    float fb, fr;           // b and r
    float step, t_stop, w_min;
};

struct CubePos {
    int64_t k;     // cube (< 0: empty cell)
    int32_t v0;    // local index of the cell corner nearest the origin
    float wx, wy, wz;
};

// cell / cell_k (optional): the last cell looked up and its index entry;
// consecutive samples in one cell then skip the dependent index read.
__device__ __forceinline__ CubePos cube_pos(const CubesC& C, float x, float y, float z, int32_t* cell = nullptr,
                                            int32_t* cell_k = nullptr) {
    const float gx = x * C.fb, gy = y * C.fb, gz = z * C.fb;
    const int cx = min(int(gx), C.b - 1), cy = min(int(gy), C.b - 1), cz = min(int(gz), C.b - 1);
    CubePos p;
    const int32_t lin = (cz * C.b + cy) * C.b + cx;
    int32_t k;
    if (cell && *cell == lin) {
        k = *cell_k;
    } else {
        k = C.index[lin];
        if (cell) {
            *cell = lin;
            *cell_k = k;
        }
    }
    p.k = k < 0 ? -1 : min<int64_t>(k, C.n_cubes - 1);  // an entry past the table reads its last cube
    const float ux = (gx - float(cx)) * C.fr, uy = (gy - float(cy)) * C.fr, uz = (gz - float(cz)) * C.fr;
    const int px = min(int(ux), C.r - 1), py = min(int(uy), C.r - 1), pz = min(int(uz), C.r - 1);
    p.wx = ux - float(px);
    p.wy = uy - float(py);
    p.wz = uz - float(pz);
    p.v0 = (pz * C.r1 + py) * C.r1 + px;
    return p;
}

// Trilinear weight of corner c = dx + 2 dy + 4 dz.
__device__ __forceinline__ float corner_weight(const CubePos& p, int c) {
    return ((c & 1) ? p.wx : 1.f - p.wx) * ((c & 2) ? p.wy : 1.f - p.wy) * ((c & 4) ? p.wz : 1.f - p.wz);
}

__device__ __forceinline__ int corner_offset(int r1, int c) {
    return ((c >> 2) & 1) * r1 * r1 + ((c >> 1) & 1) * r1 + (c & 1);
}

__device__ __forceinline__ float density_at(const CubesC& C, const CubePos& p) {
    const __half* v = C.dens + p.k * (int64_t(C.r1) * C.r1 * C.r1) + p.v0;
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += corner_weight(p, c) * __half2float(v[corner_offset(C.r1, c)]);
    return s;
}

__device__ __forceinline__ float4 diffuse_at(const CubesC& C, const CubePos& p) {
    const __half* v = C.diff + 4 * (p.k * (int64_t(C.r1) * C.r1 * C.r1) + p.v0);
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const float w = corner_weight(p, c);
        const uint2 raw = *reinterpret_cast<const uint2*>(v + 4 * corner_offset(C.r1, c));
        const __half2 lo = *reinterpret_cast<const __half2*>(&raw.x), hi = *reinterpret_cast<const __half2*>(&raw.y);
        s.x += w * __low2float(lo);
        s.y += w * __high2float(lo);
        s.z += w * __low2float(hi);
        s.w += w * __high2float(hi);
    }
    return s;
}

// Exit t along the ray of the cell of a grid of res^3 cells (fres = res)
// that holds (x, y, z): far faces; an axis the ray does not move along never
// exits.
__device__ __forceinline__ float cell_exit(int res, float fres, float3 o, float3 d, float3 inv, float x, float y,
                                           float z) {
    const float gx = x * fres, gy = y * fres, gz = z * fres;
    const int cx = min(int(gx), res - 1), cy = min(int(gy), res - 1), cz = min(int(gz), res - 1);
    const float ib = 1.f / fres;
    const float ex = d.x > 0.f ? (float(cx + 1) * ib - o.x) * inv.x : (d.x < 0.f ? (float(cx) * ib - o.x) * inv.x : INFINITY);
    const float ey = d.y > 0.f ? (float(cy + 1) * ib - o.y) * inv.y : (d.y < 0.f ? (float(cy) * ib - o.y) * inv.y : INFINITY);
    const float ez = d.z > 0.f ? (float(cz + 1) * ib - o.z) * inv.z : (d.z < 0.f ? (float(cz) * ib - o.z) * inv.z : INFINITY);
    return fminf(ex, fminf(ey, ez));
}

struct MarchArgs {
    float* rgba;     // hits: diffuse RGB and tint (completed by the shading kernel); misses: 0
    float* depth;    // nullable: t of the hit sample, +inf for misses
    float* alpha_c;  // nullable: coarse opacity of every ray (0 outside the cube)
    HitRec* tmp;     // hit records of workgroup b at blk[b].y; pad holds alpha_c's bits
    int2* blk;
    const uint8_t* macro;  // nullable: occupancy of the (b/kMacro)^3 macro cells
};

// Macro cells of kMacro^3 base cells: one flag each, set when any of its
// base cells holds a cube.  An empty macro cell is skipped in one jump.
constexpr int kMacro = 4;

__global__ void k_cube_macro(const int32_t* __restrict__ index, int b, uint8_t* __restrict__ macro) {
    const int bm = b / kMacro;
    const int m = int(blockIdx.x) * blockDim.x + threadIdx.x;
    if (m >= bm * bm * bm) return;
    const int mx = m % bm, my = (m / bm) % bm, mz = m / (bm * bm);
    uint8_t any = 0;
    for (int k = 0; k < kMacro * kMacro * kMacro; ++k) {
        const int cx = mx * kMacro + k % kMacro, cy = my * kMacro + (k / kMacro) % kMacro,
                  cz = mz * kMacro + k / (kMacro * kMacro);
        any |= index[(int64_t(cz) * b + cy) * b + cx] >= 0 ? 1 : 0;
    }
    macro[m] = any;
}

__global__ __launch_bounds__(kThreads) void k_march(CubesC C, CamC cam, MarchArgs a) {
    __shared__ int s_cnt[kThreads / 64];
    const int lane = __lane_id(), wave = int(threadIdx.x) / 64;
    int tx, ty;
    tile_at(int(blockIdx.x), cam.tiles_x, (cam.H + kTile - 1) / kTile, tx, ty);
    const int row = ty * kTile + 8 * (wave >> 1) + (lane >> 3), col = tx * kTile + 8 * (wave & 1) + (lane & 7);
    const bool valid = row < cam.H && col < cam.W;
    const int64_t ray = int64_t(row) * cam.W + col;
    const int64_t base = int64_t(ty) * kTile * cam.W + int64_t(tx) * kTile * min(kTile, cam.H - ty * kTile);
    const float3 d = camera_dir(cam, row, col);
    const float3 o = make_float3(cam.o[0], cam.o[1], cam.o[2]);
    const float3 inv = make_float3(1.f / d.x, 1.f / d.y, 1.f / d.z);
    // the ray inside [0,1]^3
    float t_in = 0.f, t_out = INFINITY;
    {
        const float oo[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z}, ii[3] = {inv.x, inv.y, inv.z};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (dd[k] == 0.f) {
                if (!(oo[k] >= 0.f && oo[k] <= 1.f)) t_out = -INFINITY;
            } else {
                const float t0 = (0.f - oo[k]) * ii[k], t1 = (1.f - oo[k]) * ii[k];
                t_in = fmaxf(t_in, fminf(t0, t1));
                t_out = fminf(t_out, fmaxf(t0, t1));
            }
        }
    }
    const bool finite = isfinite(o.x) && isfinite(o.y) && isfinite(o.z) && isfinite(d.x) && isfinite(d.y) &&
                        isfinite(d.z);
    float best_w = 0.f, best_t = INFINITY, ac = 0.f, T = 1.f;
    float3 best_x = make_float3(0.f, 0.f, 0.f);
    if (valid && finite && t_in < t_out) {
        int32_t cell = -1, cell_k = -1, mcell = -1;
        const int bm = C.b / kMacro;
        const float fbm = float(bm);
        for (int j = 0; j < C.j_max;) {
            const float t = t_in + (float(j) + 0.5f) * C.step;
            if (!(t < t_out)) break;
            const float x = clamp01(o.x + t * d.x), y = clamp01(o.y + t * d.y), z = clamp01(o.z + t * d.z);
            if (a.macro) {
                const int mx = min(int(x * fbm), bm - 1), my = min(int(y * fbm), bm - 1), mz = min(int(z * fbm), bm - 1);
                const int m = (mz * bm + my) * bm + mx;
                if (m != mcell) {  // a macro cell already found occupied is not read again
                    if (!a.macro[m]) {
                        const float q = (cell_exit(bm, fbm, o, d, inv, x, y, z) - t_in) / C.step - 0.5f;
                        const float jn = ceilf(q - 0.01f);
                        j = jn > float(j + 1) ? (jn < float(C.j_max) ? int(jn) : C.j_max) : j + 1;
                        continue;
                    }
                    mcell = m;
                }
            }
            const CubePos p = cube_pos(C, x, y, z, &cell, &cell_k);
            if (p.k < 0) {
                const float q = (cell_exit(C.b, C.fb, o, d, inv, x, y, z) - t_in) / C.step - 0.5f;
                const float jn = ceilf(q - 0.01f);
                j = jn > float(j + 1) ? (jn < float(C.j_max) ? int(jn) : C.j_max) : j + 1;
                continue;
            }
            const float sigma = density_at(C, p);
            const float em = expm1f(-sigma * C.step);  // -alpha
            const float w = T * -em;
            if (w > best_w) {
                best_w = w;
                best_t = t;
                best_x = make_float3(x, y, z);
            }
            ac += w;
            T *= expf(-sigma * C.step);
            if (T < C.t_stop) break;
            ++j;
        }
    }
    const bool hit = valid && best_w > 0.f && best_w >= C.w_min;  // an empty march never hits
    float4 diff = make_float4(0.f, 0.f, 0.f, 0.f);
    if (hit) diff = diffuse_at(C, cube_pos(C, best_x.x, best_x.y, best_x.z));
    if (valid) {
        if (a.depth) a.depth[ray] = hit ? best_t : INFINITY;
        if (a.alpha_c) a.alpha_c[ray] = ac;
        reinterpret_cast<float4*>(a.rgba)[ray] = diff;
    }
    const uint64_t mask = __ballot(hit);
    if (lane == 0) s_cnt[wave] = __popcll(mask);
    __syncthreads();
    int before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        before += w < wave ? s_cnt[w] : 0;
        total += s_cnt[w];
    }
    if (hit) {
        const int64_t pos = base + before + __popcll(mask & ((uint64_t(1) << lane) - 1));
        HitRec h;
        h.x = best_x.x;
        h.y = best_x.y;
        h.z = best_x.z;
        h.out = int32_t(ray);
        h.dx = d.x;
        h.dy = d.y;
        h.dz = d.z;
        h.pad = __float_as_int(ac);
        a.tmp[pos] = h;
    }
    if (threadIdx.x == 0) a.blk[blockIdx.x] = make_int2(total, int(base));
}

// The shading stage of the i-NOLF form on caller hit points (one thread per
// point): the diffuse colour and tint at x (zero in an empty base cell) go to
// rgba, and a hit record (x, unit direction, alpha_c in the pad) to recs in
// input order, for k_shade<..., NOLF>.  Thread 0 writes the record count.
__global__ __launch_bounds__(kThreads) void k_nolf_points(CubesC C, const float* __restrict__ x,
                                                          const float* __restrict__ d, const float* __restrict__ ac,
                                                          int64_t n, float* __restrict__ rgba,
                                                          HitRec* __restrict__ recs, int32_t* __restrict__ counter) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i == 0) *counter = int32_t(n);
    if (i >= n) return;
    const float px = clamp01(x[3 * i]), py = clamp01(x[3 * i + 1]), pz = clamp01(x[3 * i + 2]);
    const CubePos p = cube_pos(C, px, py, pz);
    reinterpret_cast<float4*>(rgba)[i] = p.k < 0 ? make_float4(0.f, 0.f, 0.f, 0.f) : diffuse_at(C, p);
    const float dx = d[3 * i], dy = d[3 * i + 1], dz = d[3 * i + 2];
    const float inv = 1.f / sqrtf(dx * dx + dy * dy + dz * dz);
    recs[i] = HitRec{px, py, pz, int32_t(i), dx * inv, dy * inv, dz * inv, __float_as_int(ac[i])};
}

}  // namespace dev
}  // namespace inrf
