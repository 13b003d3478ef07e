/*
 * inrf.h -- C ABI of an MI355X (gfx950) implementation of the i-NOLF
 * one-query-per-ray render path (Luo et al., "NEPHELE: A Neural Platform for
 * Highly Realistic Cloud Radiance Rendering", arXiv 2303.04086).
 *
 * Per ray the path finds the hit point on a triangle-mesh geometry proxy,
 * looks up multi-level features through perfect spatial hash tables with
 * trilinear blending (Sec. 4.1, Eq. 1), encodes the view direction with real
 * spherical harmonics of bands 0..3, and evaluates a small MLP that gives the
 * colour and opacity of the local opacity light field (Sec. 4.2, Eqs. 2-3).
 *
 * Conventions for every call:
 *   - Status codes: INRF_OK (0) or a negative INRF_E_* value; the message of
 *     the last failure on the calling thread is returned by inrf_last_error().
 *   - Arguments are validated before anything is enqueued; on an error no
 *     work is enqueued and no output is written.
 *   - "device" pointers are HIP device memory owned by the caller; "host"
 *     pointers are ordinary process memory owned by the caller, consumed
 *     before the call returns.  Device calls never allocate, never free and
 *     never synchronise: they enqueue on `stream` (a hipStream_t; NULL = the
 *     null stream) and return; results are valid once the caller has
 *     synchronised that stream.  Device faults surface at that point.
 *   - No C++ exception crosses this boundary.  Calls are reentrant; calls on
 *     different streams may run concurrently if they do not share output or
 *     workspace memory.
 *   - Misses (including rays with a non-finite origin or direction, or a zero
 *     direction) are defined outputs, not errors: RGBA (0,0,0,0), t = +inf,
 *     triangle -1.
 */
#ifndef INRF_H
#define INRF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t inrf_status;

#define INRF_OK 0
#define INRF_E_INVALID (-1)     /* bad argument, shape or layout; nothing enqueued */
#define INRF_E_SIZE (-2)        /* caller buffer or workspace too small */
#define INRF_E_BUILD (-3)       /* a host build did not succeed within its limits */
#define INRF_E_DEVICE (-4)      /* HIP runtime or launch error */
#define INRF_E_UNSUPPORTED (-5) /* combination not compiled in */

/* Element types of feature tables and low-precision weight copies. */
#define INRF_F32 0
#define INRF_F16 1
#define INRF_BF16 2

/* Arithmetic of the network evaluation. */
#define INRF_PREC_FP32 0 /* FP32 operands, FP32 matrix cores, FP32 accumulation */
#define INRF_PREC_FP16 1 /* FP16 operands on matrix cores, FP32 accumulation */
#define INRF_PREC_BF16 2 /* BF16 operands on matrix cores, FP32 accumulation */

#define INRF_MAX_LEVELS 32
#define INRF_FEATURES 2  /* features per level (F) */
#define INRF_SH_DIM 16   /* real SH bands 0..3 */
#define INRF_HIDDEN 64   /* width of both hidden layers */
#define INRF_OUT 4       /* R, G, B, alpha */
#define INRF_MAX_OBJECTS 16 /* objects of one scene render */
#define INRF_MAX_CAMERAS 16 /* cameras of one batched render */

/* Thread-local message of the last failed call ("" if none). */
const char* inrf_last_error(void);
/* Library version, major * 10000 + minor * 100 + patch. */
int32_t inrf_version(void);

/* ------------------------------------------------------------------------
 * Host-side builders.  Synchronous, deterministic (independent of the
 * thread count), touch no device memory.
 * ---------------------------------------------------------------------- */

/* Parameters of the perfect-spatial-hash build (Sec. 4.1: the offset table is
 * precomputed from an occupancy field with a heuristic that favours mapping
 * neighbouring points to neighbouring slots).
 *   seed          seeds the pseudo-random candidate offsets
 *   dilate        occupied cells = cells within this Chebyshev distance of a
 *                 cell whose closed box meets a proxy triangle (>= 0)
 *   load_pct      table side mbar = smallest with load_pct*mbar^3 >= 100*n
 *                 (1..100)
 *   bucket_keys   offset-table side rbar starts at the smallest value with
 *                 bucket_keys*rbar^3 >= n (>= 1), then grows until
 *                 gcd(mbar, rbar) = 1 and mbar*rbar >= N+1
 *   n_random      pseudo-random candidate offsets tried per bucket
 *   max_restarts  rbar increases before mbar is increased
 *   n_threads     worker threads for voxelisation (0 = hardware count) */
typedef struct inrf_psh_params {
    uint64_t seed;
    int32_t dilate;
    int32_t load_pct;
    int32_t bucket_keys;
    int32_t n_random;
    int32_t max_restarts;
    int32_t n_threads;
} inrf_psh_params;

/* Fills the defaults: seed 1, dilate 1, load_pct 80, bucket_keys 2,
 * n_random 32, max_restarts 4, n_threads 0. */
void inrf_psh_params_default(inrf_psh_params* p);

typedef struct inrf_psh inrf_psh; /* opaque host object */

typedef struct inrf_psh_level_info {
    int32_t res;      /* grid resolution N (cells per axis; vertices 0..N) */
    int32_t mbar;     /* hash table side: mbar^3 slots */
    int32_t rbar;     /* offset table side: rbar^3 entries */
    int32_t restarts; /* rebuilds needed (rbar or mbar increases) */
    int64_t n_keys;   /* occupied vertices */
    int64_t n_slots;  /* mbar^3 */
    int64_t n_phi;    /* rbar^3 */
} inrf_psh_level_info;

/* Voxelise the proxy at each resolution res[l] (occupied vertices of Sec. 4.2,
 * "Implementation with PSH encoding"), then build each level's offset table
 * Phi and key->slot map (Sec. 4.1, Eq. 1):
 *     slot(p) = (p + Phi[p mod rbar]) mod mbar   (component-wise),
 *     linear slot = (s_z*mbar + s_y)*mbar + s_x.
 * verts: host float32 [n_verts][3], every coordinate in [0,1] and a multiple
 * of 2^-16 (so occupancy is decided exactly in integers); tris: host int32
 * [n_tris][3] vertex indices.  res: host int32 [n_levels], each in
 * [1, 4096].  On success *out owns the result (free with inrf_psh_free).
 * Errors: INRF_E_INVALID (bad sizes, vertex off the 2^-16 lattice or outside
 * [0,1], index out of range), INRF_E_BUILD (mbar would exceed 1024). */
inrf_status inrf_build_psh(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                           int32_t n_levels, const int32_t* res, const inrf_psh_params* params,
                           inrf_psh** out);

/* Build one level from a caller-supplied occupied vertex set (for occupancy
 * that does not come from a mesh, e.g. shape from silhouette).
 * keys: host int64 [n_keys] linear vertex keys (z*(N+1)+y)*(N+1)+x, strictly
 * ascending.  params->dilate is ignored. */
inrf_status inrf_build_psh_keys(int32_t res, const int64_t* keys, int64_t n_keys,
                                const inrf_psh_params* params, inrf_psh** out);

/* Number of levels of a built object. */
int32_t inrf_psh_levels(const inrf_psh* psh);

/* Copy one level out.  info is required; keys (int64 [n_keys], canonical
 * ascending linear keys), phi (uint32 [n_phi], packed x | y<<10 | z<<20) and
 * slots (int32 [n_keys], linear slot of each key in key order) are optional
 * host buffers of the sizes given by info. */
inrf_status inrf_psh_level(const inrf_psh* psh, int32_t level, inrf_psh_level_info* info,
                           int64_t* keys, uint32_t* phi, int32_t* slots);

void inrf_psh_free(inrf_psh* psh);

/* Device storage order of a level's two cubes (the hash table H of side mbar
 * and the offset table Phi of side rbar).  Cells are stored in bricks of
 * 8 x 4 x 1 cells (32 entries, one 128-byte line of 4-byte entries), x
 * fastest inside a brick and across bricks, each z plane padded to whole
 * bricks:
 *   index(x, y, z) = z * P + (y/4) * R + (x/8) * 32 + (y%4) * 8 + x%8,
 *   R = 32 * ceil(side/8), P = R * ceil(side/4),
 * so the eight corners of a cell span 2.8 lines on average instead of 4.1.
 * The slot of Eq. 1 is unchanged; only where it is stored differs.
 * inrf_brick_entries: entries one level's cube occupies (P * side), -1 if
 * side is not in [1, 1024].  inrf_brick_index: storage index of each linear
 * cell index (z*side + y)*side + x (host arrays of n; INRF_E_INVALID if one
 * is out of range, then nothing is written). */
int64_t inrf_brick_entries(int32_t side);
inrf_status inrf_brick_index(int32_t side, const int64_t* linear, int64_t n, int64_t* out);

typedef struct inrf_bvh inrf_bvh; /* opaque host object */

typedef struct inrf_bvh_info {
    int64_t n_nodes;    /* four-wide nodes */
    int64_t node_bytes; /* size of the node image */
    int64_t tri_bytes;  /* size of the triangle image */
    int32_t depth;      /* deepest leaf (root = 1) */
    int32_t max_leaf;   /* triangles per leaf, at most 4 */
    int32_t stack;      /* traversal stack entries a ray can need (1..64) */
    int32_t pad;
} inrf_bvh_info;

/* Bounding volume hierarchy over the proxy (the paper queries a geometry
 * proxy per ray, abstract and Sec. 1; this is its acceleration structure):
 * binned SAH, then collapsed to four-wide nodes.  Same vertex/triangle arguments as inrf_build_psh, except that
 * coordinates need not lie on the lattice (they must be finite). */
inrf_status inrf_build_bvh(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                           inrf_bvh** out);
inrf_status inrf_bvh_get_info(const inrf_bvh* bvh, inrf_bvh_info* info);
/* Copy the node and triangle images (opaque layouts) into host buffers of
 * info.node_bytes and info.tri_bytes; the caller uploads them to the device
 * and points inrf_model at them. */
inrf_status inrf_bvh_copy(const inrf_bvh* bvh, void* nodes, void* tri_data);
void inrf_bvh_free(inrf_bvh* bvh);

/* ------------------------------------------------------------------------
 * Device model: a plain view of caller-owned device memory.
 * ---------------------------------------------------------------------- */

typedef struct inrf_level_desc {
    int32_t res, mbar, rbar, pad;
    int64_t phi_offset;  /* first entry of this level in `phi` (inrf_brick_entries(rbar) entries) */
    int64_t slot_offset; /* first entry of this level in `table` (inrf_brick_entries(mbar) entries) */
} inrf_level_desc;

typedef struct inrf_model {
    int32_t n_levels;    /* L, 1..INRF_MAX_LEVELS */
    int32_t table_dtype; /* INRF_F32 or INRF_F16 */
    inrf_level_desc levels[INRF_MAX_LEVELS];
    const uint32_t* phi;    /* device, packed offsets of all levels, each level's cube
                               in the brick order of inrf_brick_index */
    const void* table;      /* device, [total entries][INRF_FEATURES] of table_dtype,
                               each level's cube in brick order; slots of unoccupied
                               vertices and padding hold zeros */
    const float* weights;   /* device FP32 W1 [64][d_in] | W2 [64][64] | W3 [4][64],
                               row-major [out][in], d_in = 2*L + 16; the FP16 and
                               BF16 precisions round them on the fly */
    const void* bvh_nodes;  /* device image from inrf_bvh_copy */
    const void* bvh_tris;   /* device image from inrf_bvh_copy */
    int64_t n_tris;         /* proxy triangles; 0 = empty proxy (every ray misses) */
    int32_t bvh_stack;      /* inrf_bvh_info.stack of the image (sizes the traversal stack) */
    int32_t bvh_n_nodes;    /* inrf_bvh_info.n_nodes of the image */
} inrf_model;

/* Pinhole camera (pose and intrinsics as a client sends them).  Pixel (i
 * from the top, j from the left) of a width x height image has ray index
 * i*width + j, origin `origin` and direction
 *     normalize(forward + s_x*right + s_y*up),
 *     s_x = (2(j+1/2)/width - 1) * tan_half_fov_y * width/height,
 *     s_y = (1 - 2(i+1/2)/height) * tan_half_fov_y. */
typedef struct inrf_camera {
    float origin[3], right[3], up[3], forward[3];
    float tan_half_fov_y;
    int32_t width, height;
} inrf_camera;

/* Workspace bytes needed by inrf_render / inrf_forward for up to n_rays rays. */
int64_t inrf_workspace_size(int64_t n_rays);

/* Render one camera (the clients of the rendering service send a camera pose
 * and intrinsics per frame, Sec. 5; every pixel is one ray, Sec. 1): rgba
 * (device float32 [height*width][4], row-major, top
 * row first, not premultiplied), and optionally depth (device float32
 * [height*width], distance along the unit ray, +inf on a miss) and tri
 * (device int32 [height*width], proxy triangle index, -1 on a miss).
 * ws: device workspace of at least inrf_workspace_size(width*height) bytes;
 * its first two int32 receive the frame's hit-ray count and zero.  The
 * proxy's triangles are first sorted into lists per 8x8-pixel quadrant of
 * the frame (256 slots per quadrant, longer lists in a spill area of one
 * entry per pixel; a quadrant whose list fits neither is traced through the
 * BVH instead), and
 * every ray is tested against its quadrant's list: the closest hit (ties to
 * the lower triangle index) is the one inrf_forward finds on the same ray
 * through the BVH.  Everything is enqueued on `stream`. */
inrf_status inrf_render(const inrf_model* m, int32_t precision, const inrf_camera* cam, float* rgba,
                        float* depth, int32_t* tri, void* ws, int64_t ws_bytes, void* stream);

/* The primary rays of a camera (one ray per pixel from the pose a client
 * sends, Sec. 5) exactly as the render kernels generate them: ray_o
 * (nullable) and ray_d device float32
 * [height*width][3], row-major, unit directions.  inrf_forward on these
 * rays gives every pixel exactly the value inrf_render gives it. */
inrf_status inrf_camera_rays(const inrf_camera* cam, float* ray_o, float* ray_d, void* stream);

/* inrf_render with stage timing: events (host array of 3 hipEvent_t created
 * by the caller; NULL entries are skipped) are recorded on `stream` before
 * the trace, between the trace and the shading, and after the shading, so
 * the caller can measure each stage with hipEventElapsedTime. */
inrf_status inrf_render_profiled(const inrf_model* m, int32_t precision, const inrf_camera* cam, float* rgba,
                                 float* depth, int32_t* tri, void* ws, int64_t ws_bytes, void* stream,
                                 void* const* events);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * inrf_render without a workspace argument.  Its scratch memory is a static
 * device array of the library (75.9 MiB, held by each GPU the library
 * runs on until the process ends), so frames are limited to
 * INRF_STATIC_MAX_PIXELS pixels (INRF_E_SIZE beyond, nothing enqueued).
 * The call allocates nothing and creates no runtime object.  Every call on
 * one GPU shares that array: calls
 * that may overlap on one GPU (different streams without ordering between
 * them, or several host threads) race and must be serialised by the
 * caller.  Nothing in the array needs to start at zero: every value a
 * frame reads was written earlier in the same frame.  Pixels are exactly
 * those inrf_render gives. */
#define INRF_STATIC_MAX_PIXELS 1048576
inrf_status inrf_render_static(const inrf_model* m, int32_t precision, const inrf_camera* cam, float* rgba,
                               float* depth, int32_t* tri, void* stream);

/* The same path on a batch of rays ("an indiscriminate range of rays with
 * depths", Sec. 1): ray_o, ray_d device float32 [n][3] (d need not be unit;
 * depth is then the ray parameter t); rgba device float32 [n][4]; depth and
 * tri optional as in inrf_render. */
inrf_status inrf_forward(const inrf_model* m, int32_t precision, const float* ray_o, const float* ray_d,
                         int64_t n, float* rgba, float* depth, int32_t* tri, void* ws, int64_t ws_bytes,
                         void* stream);

/* Several cameras in one pass (the requests of several clients, Sec. 6,
 * traced and shaded together: one trace launch over all their tiles and one
 * shading launch over all their hit rays).  cams: host array of n_cameras
 * (1..INRF_MAX_CAMERAS); rgba (and depth, tri if set) hold the images one
 * after another in camera order, each as inrf_render writes it.  Every
 * pixel gets exactly the value inrf_render gives it.  ws: at least
 * inrf_batch_workspace_size(n_cameras, total pixels) bytes. */
int64_t inrf_batch_workspace_size(int32_t n_cameras, int64_t n_pixels);
inrf_status inrf_render_batch(const inrf_model* m, int32_t precision, const inrf_camera* cams, int32_t n_cameras,
                              float* rgba, float* depth, int32_t* tri, void* ws, int64_t ws_bytes, void* stream);

/* Closest hit only: tri (device int32 [n]) and t (device float32 [n]). */
inrf_status inrf_trace(const inrf_model* m, const float* ray_o, const float* ray_d, int64_t n, int32_t* tri,
                       float* t, void* stream);

/* Position encoding E(x) (Sec. 4.1): x device float32 [n][3] (clamped to
 * [0,1]); enc device float32 [n][2L], level 0 first; slots optional device
 * int32 [n][L][8] (level-local linear slot of corner c = cx + 2cy + 4cz). */
inrf_status inrf_encode(const inrf_model* m, const float* x, int64_t n, float* enc, int32_t* slots,
                        void* stream);

/* The network alone (Sec. 4.2, Eq. 3): in device float32 [n][d_in] (encoding
 * then 16 SH values), rgba device float32 [n][4]. */
inrf_status inrf_mlp(const inrf_model* m, int32_t precision, const float* in, int64_t n, float* rgba,
                     void* stream);

/* The network on 16-bit inputs (Sec. 4.2, Eq. 3): enc device [n][2L]
 * encodings of the precision's 16-bit type (INRF_PREC_FP16: IEEE half,
 * INRF_PREC_BF16: bfloat16), dir device float32 [n][3] view directions
 * (need not be unit); the SH16 values of dir / |dir| are computed on the
 * fly, as the shading kernel does.  rgba device float32 [n][4], 16-byte
 * aligned.  INRF_PREC_FP32 is refused (INRF_E_INVALID): use inrf_mlp. */
inrf_status inrf_mlp_encoded(const inrf_model* m, int32_t precision, const void* enc, const float* dir, int64_t n,
                             float* rgba, void* stream);

/* ------------------------------------------------------------------------
 * Scenes of several objects (the paper composes objects per pixel by depth,
 * Sec. 5; scenes of several objects, Sec. 7).
 * ---------------------------------------------------------------------- */

/* One object of a scene: its model (host pointer to the model view, whose
 * device memory must stay valid until the render completes) placed in the
 * world by a similarity transform
 *     x_world = scale * rotation * x_object + translation,
 * scale > 0, rotation row-major, orthonormal with determinant +1. */
typedef struct inrf_instance {
    const inrf_model* model;
    float scale;
    float rotation[9];
    float translation[3];
} inrf_instance;

/* Workspace bytes inrf_render_scene needs for n_objects and n_rays pixels;
 * -1 on invalid arguments. */
int64_t inrf_scene_workspace_size(int32_t n_objects, int64_t n_rays);

/* Render one camera over a scene of n_objects (0..INRF_MAX_OBJECTS) objects
 * (the per-pixel depth composition of objects of Sec. 5, in one pass):
 * per pixel the nearest hit over all objects wins (equal distance: the lower
 * object index), and that object's network shades it from the object-space
 * hit point and direction.  rgba as inrf_render; depth (nullable) is the
 * world distance along the unit ray; tri (nullable) the triangle of the
 * winning object's proxy; object (nullable, device int32 [height*width]) the
 * winning object's index, -1 on a miss.  Every object's model uses the same
 * precision; tables may differ in type.  ws: 256-byte aligned, at least
 * inrf_scene_workspace_size(n_objects, width*height) bytes. */
inrf_status inrf_render_scene(const inrf_instance* objects, int32_t n_objects, int32_t precision,
                              const inrf_camera* cam, float* rgba, float* depth, int32_t* tri, int32_t* object,
                              void* ws, int64_t ws_bytes, void* stream);

/* Several cameras over one scene in one pass (the requests of several
 * clients of a resident scene, Sec. 6, with the per-pixel depth composition
 * of Sec. 5): one trace launch over all the cameras' tiles, then one
 * shading launch per object over that object's hit rays from every camera.
 * cams: host array of n_cameras (1..INRF_MAX_CAMERAS); rgba (and depth,
 * tri, object if set) hold the images one after another in camera order,
 * each as inrf_render_scene writes it, and every pixel gets exactly the
 * value inrf_render_scene gives it.  ws: 256-byte aligned, at least
 * inrf_scene_batch_workspace_size(n_objects, n_cameras, total pixels)
 * bytes (-1 on invalid arguments). */
int64_t inrf_scene_batch_workspace_size(int32_t n_objects, int32_t n_cameras, int64_t n_pixels);
inrf_status inrf_render_scene_batch(const inrf_instance* objects, int32_t n_objects, int32_t precision,
                                    const inrf_camera* cams, int32_t n_cameras, float* rgba, float* depth,
                                    int32_t* tri, int32_t* object, void* ws, int64_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * The paper's own i-NOLF form (Sec. 4.2): the hit point comes from a march
 * through cached density texture cubes (Eq. 4, the sample of largest
 * weight), the summed weights (coarse opacity alpha_c) are a further input
 * of the network, which returns the specular colour c_s and the opacity,
 * and cached diffuse texture cubes give the diffuse colour c_d and the
 * specular tint t at the hit: colour = c_d + t * c_s (Eq. 6-7).
 * ---------------------------------------------------------------------- */

/* Texture cubes: a base grid of b^3 cells, each holding the index of a small
 * dense cube of (r+1)^3 vertex values over the cell, or a negative value
 * (empty: density 0).  The value at x in [0,1]^3 is the trilinear blend of
 *   g = b x, c = min(floor(g), b-1), u = (g - c) r, p = min(floor(u), r-1)
 * over the cube's vertices p + {0,1}^3.  Density and diffuse cubes share the
 * index.  All pointers are caller-owned device memory. */
typedef struct inrf_cubes {
    int32_t base_res;      /* b: a power of two in [1, 1024] */
    int32_t cube_res;      /* r: a power of two in [1, 64] */
    const int32_t* index;  /* [b^3], cell (cz*b + cy)*b + cx; entries >= n_cubes read the last cube */
    const void* density;   /* FP16 [n_cubes][(r+1)^3], vertex (i, j, k) at (k*(r+1) + j)*(r+1) + i */
    const void* diffuse;   /* FP16 [n_cubes][(r+1)^3][4]: diffuse R, G, B, tint; 8-byte aligned */
    int64_t n_cubes;       /* >= 1 */
    float step;            /* march step in object units, in [1e-6, 1] (e.g. sqrt(3)/1024) */
    float t_stop;          /* the march ends once transmittance falls below this, in (0, 1) (e.g. 1e-4) */
    float w_min;           /* a ray hits if its largest sample weight is at least this, in (0, 1] (e.g. 1e-4);
                              a march that meets no density never hits */
    int32_t pad;
} inrf_cubes;

/* Render one camera with the i-NOLF form (Sec. 4.2, Eqs. 4-7).  The ray (unit direction) is
 * marched inside [0,1]^3 at t_in + (j + 1/2) step; each sample's density s
 * gives alpha = 1 - exp(-s step), weight w = T alpha and T *= exp(-s step);
 * the march ends after the first sample whose T falls below t_stop.  The
 * hit is the sample of largest weight (the first on ties) if that weight is
 * at least w_min, else the ray misses.  m supplies the level tables and the
 * weights, whose first layer takes d_in = 2L + 17 inputs: the encoding,
 * SH16 of the direction, then alpha_c; its proxy fields are ignored; at most
 * 8 levels.  rgba (16-byte aligned, [height*width][4]): hits
 * (c_d + t c_s, alpha), misses 0.  depth (nullable): t of the hit sample,
 * +inf on a miss.  alpha_c (nullable): the summed weights of every ray.
 * ws: 256-byte aligned, at least inrf_workspace_size(width*height) bytes. */
inrf_status inrf_render_nolf(const inrf_model* m, const inrf_cubes* cubes, int32_t precision,
                             const inrf_camera* cam, float* rgba, float* depth, float* alpha_c, void* ws,
                             int64_t ws_bytes, void* stream);

/* The shading stage of the i-NOLF form alone (Sec. 4.2, Eqs. 3, 6-7) on n
 * caller hit points: x device float32 [n][3] (clamped to [0,1]), d device
 * float32 [n][3] (need not be unit), alpha_c device float32 [n]; rgba
 * (device float32 [n][4], 16-byte aligned) = (c_d + t c_s, alpha) with c_d
 * and t read from the diffuse cubes at x (zero in an empty base cell) and
 * (c_s, alpha) from the network on (encoding of x, SH16 of d, alpha_c),
 * through the same kernel inrf_render_nolf shades its hits with.  ws:
 * 256-byte aligned, at least inrf_workspace_size(n) bytes. */
inrf_status inrf_shade_nolf(const inrf_model* m, const inrf_cubes* cubes, int32_t precision, const float* x,
                            const float* d, const float* alpha_c, int64_t n, float* rgba, void* ws, int64_t ws_bytes,
                            void* stream);

/* ------------------------------------------------------------------------
 * Gradient (training, Sec. 4.2 with the loss of Eq. 8).
 * ---------------------------------------------------------------------- */

/* Workspace bytes needed by inrf_backward for up to n_rays rays with model m
 * on the current device (the hit records plus one weight-gradient partial
 * per resident workgroup); -1 on invalid arguments. */
int64_t inrf_backward_workspace_size(const inrf_model* m, int64_t n_rays);

/* Adds the gradient of a loss L (e.g. Eq. 8's, Sec. 4.2) with respect to the model's parameters,
 * given d_rgba = dL/d(rgba) (device float32 [n][4], 16-byte aligned) for the
 * batch of rays ray_o, ray_d (as inrf_forward):
 *   d_table   device float32 [total slots][INRF_FEATURES], the layout of the
 *             model's table; gradient w.r.t. the feature of every slot the
 *             rays read, ADDED in place (FP32 atomic adds: the rounding of
 *             a slot hit by several rays depends on their order).  NULL skips
 *             it.  The table itself may be FP32 or FP16; the forward pass is
 *             recomputed from it.
 *   d_weights device float32 laid out like the model's weights (W1|W2|W3);
 *             gradient ADDED in place, deterministic.  NULL skips it.
 *   rgba      optional device float32 [n][4]: the forward output the
 *             gradient was taken at (FP32 network), written if set.
 * The network runs in FP32 (matrix cores) whatever precision inrf_forward
 * used; a missed ray contributes nothing.  Models of up to 16 levels
 * (INRF_E_UNSUPPORTED beyond).  Activations are recomputed, not
 * read from a previous forward call.  ws: device workspace, 256-byte
 * aligned, of at least inrf_backward_workspace_size(m, n) bytes. */
inrf_status inrf_backward(const inrf_model* m, const float* ray_o, const float* ray_d, int64_t n,
                          const float* d_rgba, float* d_table, float* d_weights, float* rgba, void* ws,
                          int64_t ws_bytes, void* stream);

/* One Adam step (Kingma and Ba, 2015; the optimiser of Sec. 4.2's training)
 * over n parameters, in place on device float32 arrays:
 *   m = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2,
 *   param -= lr * (m / (1 - beta1^step)) / (sqrt(v / (1 - beta2^step)) + eps).
 * With zero_grad set, g is cleared after use.  param_f16 (nullable, device
 * half [n]) receives the updated parameters rounded to FP16, e.g. the FP16
 * feature table the reduced-precision render reads.  With lazy set, only
 * parameters whose g is nonzero are stepped (and cleared, and copied to
 * param_f16); the others keep their value and moments, so a step over a
 * table of which a batch touched a small part reads g everywhere but param,
 * m and v only where g is nonzero (sparse or "lazy" Adam; step is still the
 * global step count). */
typedef struct inrf_adam_params {
    float lr, beta1, beta2, eps;
    int64_t step;      /* t >= 1 */
    int32_t zero_grad; /* nonzero: clear grad */
    int32_t lazy;      /* nonzero: step only parameters with a nonzero gradient */
} inrf_adam_params;

inrf_status inrf_adam(float* param, float* grad, float* m, float* v, int64_t n, const inrf_adam_params* p,
                      void* param_f16, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* INRF_H */
