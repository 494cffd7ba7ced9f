/*
 * vdbc — fixed-rate hierarchical (VDB) compression of dense float32 volumes
 * and GPU random-access sampling / rendering of the compressed tree on AMD
 * Instinct MI355X (gfx950).
 *
 * Method: "GPU Volume Rendering with Hierarchical Compression Using VDB"
 * (Zellmann, Jaros, Amstutz, Wald).  The encoder is Alg. 1 ("Compress",
 * Section 3.1) with the tree of Section 3.2 (8^3 leaves, 16^3-child lower
 * nodes, 32^3-child upper nodes, child/tile bit masks with popcount offsets);
 * sampling is the level-0 nearest / trilinear reconstruction of Section 3.2.2
 * with the background value where no voxel exists; rendering is the
 * emission-absorption marcher and the majorant-grid delta-tracking path tracer
 * of Section 4.
 *
 * Conventions for every call:
 *  - Every call returns a vdbc_status and never aborts.  Arguments are checked
 *    before any work is enqueued; on error nothing is enqueued and
 *    vdbc_last_error() (thread-local) holds a description.  Faults inside a
 *    kernel surface at the caller's stream synchronisation.
 *  - Device calls are stream-ordered on `stream` (a hipStream_t passed as
 *    void*; NULL = the default stream) and return once the work is enqueued.
 *  - The library allocates no device memory: every device pointer (buffer,
 *    positions, outputs, workspace) is owned by the caller and must stay valid
 *    until the enqueued work has finished.
 *  - Volumes are x-fastest: voxel (x,y,z) is element x + nx*(y + ny*z).
 *    Sample positions are in index space: voxel centres on the integers, the
 *    volume covering the box [-0.5, n-0.5] on each axis.
 */
#ifndef VDBC_H
#define VDBC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VDBC_ABI_VERSION 2u

typedef enum {
    VDBC_OK = 0,
    VDBC_E_INVALID = 1,          /* bad argument (null, size, range, NaN/Inf input) */
    VDBC_E_NOMEM = 2,            /* host allocation failed */
    VDBC_E_BUFFER_TOO_SMALL = 3, /* output capacity or workspace too small */
    VDBC_E_FORMAT = 4,           /* buffer header/structure is not format v1 */
    VDBC_E_DEVICE = 5,           /* HIP runtime error at enqueue */
    VDBC_E_UNSUPPORTED = 6
} vdbc_status;

const char* vdbc_status_string(vdbc_status s);
/* Detail of the last failing call on this thread ("" if none). */
const char* vdbc_last_error(void);
uint32_t vdbc_abi_version(void);

/* Hash (16 hex digits, static string) of the sources, header and flags the
 * library was built from.  Loaders compare it with the tree they run from
 * and refuse a stale build. */
const char* vdbc_source_hash(void);

typedef struct {
    uint32_t nx, ny, nz;
} vdbc_dims;

/* ------------------------------------------------------------------------ */
/* Host encoder: Alg. 1 (Section 3.1) + tree build and linearisation        */
/* (Section 3.2).                                                            */
/* ------------------------------------------------------------------------ */

enum {
    VDBC_BG_EXPLICIT = 1u, /* use params.background instead of the histogram mode */
    VDBC_NO_CORNERS = 2u,  /* do not force-activate the two extreme corner voxels */
    VDBC_NO_PRUNE = 4u,    /* keep uniform leaves/lower nodes instead of tiles */
    VDBC_PARTIAL = 8u      /* partial-brick activation, see vdbc_encode_params */
};

enum { VDBC_METRIC_CLOSEST = 1u, VDBC_METRIC_FARTHEST = 2u, VDBC_METRIC_MEDIAN = 3u };

typedef struct {
    float rate;         /* quality q in (0,1]: fraction of 32^3 bricks activated
                           (1:10 -> 0.10); K = min(N, floor(q*N + 0.5)) */
    uint32_t metric;    /* Eq. (1) closest, (2) farthest (default), (3) median */
    uint32_t flags;     /* VDBC_BG_EXPLICIT | VDBC_NO_CORNERS | VDBC_NO_PRUNE */
    float background;   /* used iff VDBC_BG_EXPLICIT */
    uint32_t threads;   /* host worker threads; 0 = all hardware threads */
    /* VDBC_PARTIAL only: the partial-brick activation that Section 3.2.1
     * names as future work (past a similarity threshold, a share of each
     * brick's voxels in proportionally more bricks; the paper gives no rule
     * for which voxels, this is the library's).  The
     * bricks are ranked as in Alg. 1 and K computed from `rate` as above.
     * The first F = #{ranks r < K : f_r >= partial_threshold} bricks are
     * activated whole.  The voxels plain Alg. 1 would activate in the bricks
     * ranked F..K-1 (their in-volume count R) are spent instead along the
     * bricks ranked F, F+1, ..., N-1: first ceil(partial_fraction * v_r)
     * voxels of each (v_r its in-volume voxel count; product in double),
     * then, once every such brick had that share, the rest of each brick in
     * rank order, until R voxels are active.  Inside a brick the voxels go by
     * |value - B| descending (double), ties by linear voxel index ascending.
     * So the active voxel count equals plain Alg. 1's, 1:1 stays lossless,
     * partial_fraction = 1 or a threshold below every similarity gives Alg. 1
     * itself, and the selection at a lower rate is a subset of the one at a
     * higher rate.  The header records both values (bytes 160 and 164). */
    float partial_fraction;   /* in (0, 1] */
    float partial_threshold;  /* similarity (Eq. 1-3 units), not NaN */
} vdbc_encode_params;

typedef struct {
    float background;
    uint64_t n_bricks, k_bricks, n_leaf, n_lower, n_upper, n_lower_tiles,
        n_upper_tiles, active_voxels, bytes;
    double achieved_rate; /* active voxels / (nx*ny*nz) */
} vdbc_encode_stats;

typedef struct vdbc_encoder vdbc_encoder;

/* Phase 1: analyse `dense` (host, caller-owned, x-fastest, finite values;
 * must stay unchanged until phase 2) and size the output.  On success *h is a
 * handle to pass to vdbc_encode_finish or vdbc_encode_abort, *bytes the exact
 * buffer size.  NaN/Inf input, zero dims, rate outside (0,1] or a bad metric
 * -> VDBC_E_INVALID. */
vdbc_status vdbc_encode_begin(const float* dense, vdbc_dims dims, const vdbc_encode_params* p,
                              vdbc_encoder** h, uint64_t* bytes, vdbc_encode_stats* stats);
/* Phase 2: write the canonical buffer (format v1) into host memory `out`
 * (capacity >= *bytes from phase 1, 256-byte aligned) and release the handle
 * (also on error). */
vdbc_status vdbc_encode_finish(vdbc_encoder* h, void* out, uint64_t capacity);
void vdbc_encode_abort(vdbc_encoder* h);
/* One-shot form: out == NULL or capacity too small -> VDBC_E_BUFFER_TOO_SMALL
 * with *bytes set (the analysis is then repeated by the next call). */
vdbc_status vdbc_encode(const float* dense, vdbc_dims dims, const vdbc_encode_params* p,
                        void* out, uint64_t capacity, uint64_t* bytes,
                        vdbc_encode_stats* stats);
/* Full host-side structural check of a buffer (magic, version, offsets,
 * counts, running popcount prefixes, root table). */
vdbc_status vdbc_validate(const void* buf_host, uint64_t bytes, vdbc_encode_stats* info);

/* Node layouts (header field `layout`; the encoder writes 0).  Two bits:
 * VDBC_LAYOUT_MORTON numbers the child slots of upper and lower nodes along a
 * Morton curve (bit 3b+a of a slot number = bit b of coordinate a), so lower
 * nodes, leaves and tiles are stored in Z order; VDBC_LAYOUT_SOA stores each
 * node's masks and index prefixes as four arrays (24 B per 64 slots) instead
 * of 32-byte word records.  Every layout holds the same tree.  The host calls
 * (vdbc_validate, vdbc_relayout) accept all four; the device calls read
 * layout 0 only, and vdbc_grid_init rejects the others with
 * VDBC_E_UNSUPPORTED. */
#define VDBC_LAYOUT_V1 0u
#define VDBC_LAYOUT_MORTON 1u
#define VDBC_LAYOUT_SOA 2u

/* Host.  Rewrites buffer `src` (any layout, validated first) into `layout`
 * (0..3) at `out` (host, 256-byte aligned, must not overlap `src`).  Leaf
 * masks and values are copied unchanged, nodes re-emitted in the canonical
 * order of the new slot numbering; converting back gives the original bytes.
 * out == NULL or capacity too small -> VDBC_E_BUFFER_TOO_SMALL with *bytes
 * set; a malformed source -> VDBC_E_FORMAT; layout > 3 -> VDBC_E_INVALID. */
vdbc_status vdbc_relayout(const void* src, uint64_t src_bytes, uint32_t layout, void* out,
                          uint64_t capacity, uint64_t* bytes);

/* ------------------------------------------------------------------------ */
/* Device buffer handle                                                      */
/* ------------------------------------------------------------------------ */

/* A canonical buffer resident in device memory plus a host copy of its
 * 256-byte header (the host needs dims and section offsets for launch
 * geometry without reading device memory). */
typedef struct {
    const void* device;   /* device pointer to the whole buffer, 256-B aligned */
    uint64_t bytes;
    uint8_t header[256];
} vdbc_grid;

/* Fill *g from a device pointer and the host copy of the buffer's first 256
 * bytes; checks the header (magic, version, offsets within `bytes`).  A node
 * layout other than 0 -> VDBC_E_UNSUPPORTED. */
vdbc_status vdbc_grid_init(vdbc_grid* g, const void* device, uint64_t bytes,
                           const void* host_header);

/* ------------------------------------------------------------------------ */
/* Sampling (Section 3.2.2)                                                  */
/* ------------------------------------------------------------------------ */

enum { VDBC_FILTER_NEAREST = 0u, VDBC_FILTER_TRILINEAR = 1u };

/* out[i] = field value at pos[3i..3i+2] (device float32, AoS x,y,z), for
 * i < n.  Trilinear = lerp along x, then y, then z of the 8 corner voxels,
 * B for corners outside the volume or without a voxel; nearest = voxel
 * floor(p) + (frac >= 0.5).  n == 0 is a no-op. */
vdbc_status vdbc_sample(const vdbc_grid* g, const float* pos, uint64_t n, uint32_t filter,
                        float* out, void* stream);
/* The same on a plain dense device array (the "3D texture" baseline). */
vdbc_status vdbc_sample_dense(const float* dense, vdbc_dims d, float background,
                              const float* pos, uint64_t n, uint32_t filter, float* out,
                              void* stream);
/* Integer-coordinate lookups: out[i] = value of voxel ijk[3i..3i+2] (device
 * int32; B outside the volume or where no voxel is stored). */
vdbc_status vdbc_lookup(const vdbc_grid* g, const int32_t* ijk, uint64_t n, float* out,
                        void* stream);

/* Compression error of the grid against the dense volume it approximates
 * (the MSE / PSNR evaluation of Section 5.2, tab:stats): dense = device
 * float32 of the grid's dims, x-fastest.  out = device double[5] =
 *   {sum over voxels of (vdb - dense)^2, max |vdb - dense|,
 *    voxels whose float32 bits differ, min of dense, max of dense},
 * so MSE = out[0] / voxels and a lossless grid has out[2] == 0.  ws: device
 * scratch of vdbc_compare_workspace() bytes, 8-byte aligned.  Deterministic
 * for a given size. */
vdbc_status vdbc_compare_workspace(vdbc_dims d, uint64_t* bytes);
vdbc_status vdbc_compare_dense(const vdbc_grid* g, const float* dense, double* out, void* ws,
                               uint64_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Rendering (Section 4)                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint32_t kind;          /* 0 orthographic, 1 pinhole */
    uint32_t width, height;  /* pixels; width * height <= 2^31 */
    float origin[3];        /* pinhole eye (index space) */
    float lower_left[3];    /* pinhole: direction towards image point (0,0);
                               orthographic: ray origin of image point (0,0) */
    float du[3], dv[3];     /* step per pixel along x / y of the image */
    float dir[3];           /* orthographic ray direction */
} vdbc_camera;

typedef struct {
    float sigma_scale;      /* extinction at alpha = 1 per unit of the longest
                               axis; per voxel: sigma_scale * alpha / max(n) */
    float albedo;           /* single-scattering albedo (path tracer) */
    uint32_t tf_n;          /* 2..64 RGBA control points spread evenly over */
    float tf[64][4];        /* [tf_lo, tf_hi]; alpha = extinction (Section 4) */
    float tf_lo, tf_hi;
    float light_dir[3];     /* unit vector towards the directional light */
    float light_E[3];       /* its irradiance */
    float ambient[3];       /* constant ambient radiance added on escape */
    const float* env;       /* NULL, or device float32 [env_h][env_w][3]: lat-long radiance
                               an escaping path-tracer ray sees instead of `ambient`
                               (image-based light, Section 4): nearest texel at
                               u = (atan2(d_z, d_x) + pi) / (2 pi), v = acos(d_y) / pi */
    uint32_t env_w, env_h;  /* texels (>= 1 each when env is set) */
} vdbc_medium;

enum { VDBC_MODE_EA = 0u, VDBC_MODE_PT = 1u, VDBC_MODE_ISO = 2u };
enum {
    VDBC_RENDER_HDDA = 1u,        /* EA, ISO: skip lattice samples inside empty tree
                                     nodes (result-preserving; EA needs alpha_TF(B) == 0) */
    VDBC_RENDER_COUNT = 2u,       /* count trilinear samples into the workspace */
    VDBC_RENDER_KEEP_MAJORANT = 4u, /* PT: reuse the majorant grid already in ws */
    VDBC_RENDER_RR = 8u,           /* PT: Russian roulette (Section 4): from bounce 2 on a
                                      path survives with q = min(1, max throughput) and
                                      survivors carry throughput / q; the survival draw
                                      precedes the two direction draws of each segment's
                                      stream (bounce >= 1) */
    VDBC_RENDER_CACHE_NONE = 16u,  /* PT, VDB: no per-thread cache (every lookup descends
                                      from the root) */
    VDBC_RENDER_CACHE_LEAF = 32u,  /* PT, VDB: cache the last leaf only (default, neither
                                      flag: the last leaf and the last lower node).  The
                                      image does not depend on the cache policy. */
    VDBC_RENDER_COST_ORDER = 64u   /* PT: hand the tiles to the workgroups in decreasing
                                      order of an estimated cost (the majorant optical
                                      depth of four camera rays per tile) instead of in
                                      raster order; needs 8 bytes per tile + 512 of
                                      workspace.  The image does not depend on it. */
};

typedef struct {
    uint32_t mode;          /* VDBC_MODE_EA or VDBC_MODE_PT */
    uint32_t spp;           /* PT samples per pixel, 1..65536 */
    uint32_t max_bounces;   /* PT scattering events per path, 1..65535 */
    uint32_t macrocell;     /* PT majorant cell edge in voxels: 4, 8, 16, 32 or 64 */
    uint32_t flags;         /* VDBC_RENDER_* */
    float step;             /* EA step in voxels (> 0) */
    float t_terminate;      /* EA: stop when transmittance < this (0 = off) */
    uint64_t seed;          /* PT Philox key material */
    uint32_t frame;         /* PT counter word 3 */
    uint32_t tile_w;        /* PT pixels per wave row: 8 (default; 0 = 8), 16, 32, 64;
                               a wave covers tile_w x 64 / tile_w pixels and a
                               workgroup's 256-pixel tile four of them side by side;
                               any other value -> VDBC_E_INVALID; the image does not
                               depend on it */
    float iso;              /* ISO: iso value */
    uint32_t refine;        /* ISO: bisection steps on the crossing interval (<= 64) */
    uint32_t chunk_spp;     /* PT work split: 0 or >= spp: one work item per 256-pixel
                               tile (all its samples); otherwise each tile is split into
                               ceil(spp / chunk_spp) work items of chunk_spp samples
                               (the last one shorter) that different workgroups run,
                               and the tiles' fixed-point sums meet in the workspace
                               (see below).  The image does not depend on it (integer
                               sums: bit-identical to the unsplit launch). */
} vdbc_render_params;

/* Workspace layout (caller-owned device memory, 256-B aligned):
 *   [0, 8)    uint64 trilinear-sample counter (VDBC_RENDER_COUNT; zeroed by
 *             the render call itself)
 *   [8, 16)   uint64 majorant cells visited by the path tracer's DDA (same flag)
 *   [16, 20)  uint32 path tracer work-item queue (zeroed by the render call)
 *   [24, 32)  uint64 path segments the path tracer began: camera, shadow and
 *             scattered rays (VDBC_RENDER_COUNT)
 *   [256, ..) float32 majorant grid ceil(n/macrocell)^3, x-fastest, then the
 *             coarse occupancy bits (256-B aligned)
 *   then, for a path-traced launch with 0 < chunk_spp < spp only: 40 bytes
 *             per pixel of fixed-point sums (cleared and read by the render
 *             call itself).
 * c: the camera; needed (else VDBC_E_INVALID) only when 0 < chunk_spp < spp
 * in the path tracer, may be NULL otherwise. */
vdbc_status vdbc_render_workspace(const vdbc_render_params* r, vdbc_dims d, const vdbc_camera* c,
                                  uint64_t* bytes);

/* image: device float32 [height][width][4] (RGB radiance + opacity).  aov:
 * NULL or device float32 [height][width][2] = (first-scatter depth fraction,
 * primary transmittance) for the path tracer, (hit ray parameter or -1, 0)
 * for ISO.
 * ISO (the interval-based implicit iso-surface marcher of Section 5.4): one
 * ray per pixel centre, field samples at t0 + (k + 1/2) step; the first pair
 * of consecutive samples on opposite sides of `iso` (side: f >= iso) is
 * refined by `refine` bisection steps, the hit is the midpoint of the final
 * interval and the pixel is (0.5 (n + 1), 1) with n = -grad f / |grad f|
 * from central differences of half a voxel; (0, 0, 0, 0) on a miss.  The
 * medium is not used (may be NULL).  The path tracer rebuilds the
 * majorant grid in ws first unless VDBC_RENDER_KEEP_MAJORANT. */
vdbc_status vdbc_render(const vdbc_grid* g, const vdbc_camera* c, const vdbc_medium* m,
                        const vdbc_render_params* r, float* image, float* aov, void* ws,
                        uint64_t ws_bytes, void* stream);
vdbc_status vdbc_render_dense(const float* dense, vdbc_dims d, float background,
                              const vdbc_camera* c, const vdbc_medium* m,
                              const vdbc_render_params* r, float* image, float* aov,
                              void* ws, uint64_t ws_bytes, void* stream);

/* Bytes of the fixed device scratch that vdbc_render_noalloc uses. */
#define VDBC_NOALLOC_SCRATCH_BYTES (16ull << 20)

/* vdbc_render of a VDB without a caller workspace and without any device
 * allocation, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * workspace of vdbc_render is replaced by a fixed library-owned scratch of
 * VDBC_NOALLOC_SCRATCH_BYTES (16 MiB) per GPU, held until the process ends:
 * a path-traced frame whose vdbc_render_workspace exceeds it (e.g. the
 * majorant grid of a 1987x1351x2449 volume at macrocell 8, 52 MB, or the
 * per-pixel sums of a split launch of more than about 400,000 pixels) is
 * rejected with VDBC_E_BUFFER_TOO_SMALL before anything is enqueued; use
 * vdbc_render with a workspace, a larger macrocell or chunk_spp = 0 then.  Arguments,
 * outputs and results are those of vdbc_render (bit-identical images), except
 * that VDBC_RENDER_KEEP_MAJORANT is rejected (VDBC_E_INVALID: the scratch
 * holds no majorant of the caller's).  Every call on one GPU shares its
 * scratch and each call re-initialises what it reads (counters, queue,
 * majorant, occupancy bits) on `stream`; calls that overlap on one GPU
 * (other streams, other host threads) race and must be serialised by the
 * caller.  The sample counter (VDBC_RENDER_COUNT) stays in the scratch and
 * is not readable by the caller. */
vdbc_status vdbc_render_noalloc(const vdbc_grid* g, const vdbc_camera* c, const vdbc_medium* m,
                                const vdbc_render_params* r, float* image, float* aov,
                                void* stream);

/* Majorant grid alone (Section 4 macrocells): out = device float32
 * ceil(n/macrocell)^3, x-fastest; per cell the extinction maximum over the
 * value range of voxels [C*c-1, C*c+C] (one-voxel dilation). */
vdbc_status vdbc_majorant(const vdbc_grid* g, const vdbc_medium* m, uint32_t macrocell,
                          float* out, void* stream);
vdbc_status vdbc_majorant_dense(const float* dense, vdbc_dims d, float background,
                                const vdbc_medium* m, uint32_t macrocell, float* out,
                                void* stream);

/* ------------------------------------------------------------------------ */
/* Batched rendering of many volumes (this project's extension)              */
/* ------------------------------------------------------------------------ */
typedef struct {
    vdbc_grid grid;          /* the volume (device buffer + host header copy) */
    vdbc_camera camera;
    vdbc_medium medium;
    uint32_t spp, max_bounces;  /* as in vdbc_render_params: 1..65536, 1..65535 */
    uint64_t seed;
    uint32_t frame;
    float* image;            /* device float32 [height][width][4] */
} vdbc_batch_item;

typedef struct {
    uint32_t macrocell;      /* majorant cell edge in voxels: 4, 8, 16, 32, 64 (default 16) */
    uint32_t tile_w;         /* pixels per wave row: 8, 16, 32, 64 (default 8) */
    uint32_t blocks_per_cu;  /* persistent workgroups per compute unit (default 4) */
    uint32_t persistent;     /* 1: one launch of every volume's majorant grid, one
                                of their coarse bits and one persistent render
                                launch over all (volume, work item) entries;
                                0: these launches once per volume */
    uint32_t chunk_spp;      /* samples per work item: 0 (or >= a volume's spp)
                                keeps one item per tile; 0 < chunk_spp < spp
                                splits each tile of that volume into
                                ceil(spp / chunk_spp) items whose pixels meet in
                                integer sums in the workspace (bit-identical
                                images); at most 2^20 - 1 items per volume */
} vdbc_tuning;

typedef struct vdbc_batch vdbc_batch;

/* Workspace bytes for a batch (counter, descriptor table, the prefix tables
 * of the batched majorant launches, work list, and per volume a majorant grid,
 * coarse occupancy bits and, for a volume split into work items, its pixel
 * sums).  tuning may be NULL. */
vdbc_status vdbc_batch_workspace(const vdbc_batch_item* items, uint32_t n,
                                 const vdbc_tuning* tuning, uint64_t* bytes);
/* Validates the items, uploads the descriptor table, the prefix tables and
 * the work list (volumes ordered by estimated cost, largest first; a volume's
 * tiles, or their work items, in raster order) into ws (synchronises `stream`),
 * and returns a plan.  Buffers and images must outlive the plan.  Each image
 * is bit-identical to vdbc_render of that item with the same tuning. */
vdbc_status vdbc_batch_create(const vdbc_batch_item* items, uint32_t n,
                              const vdbc_tuning* tuning, void* ws, uint64_t ws_bytes,
                              void* stream, vdbc_batch** plan);
/* Enqueues majorant builds and the render(s) on `stream`. */
vdbc_status vdbc_batch_launch(vdbc_batch* plan, void* stream);
/* Captures the launch sequence once into a HIP graph held by the plan
 * (`stream` must be a non-default, idle stream); replay it with
 * vdbc_batch_graph_launch.  No memset nodes are recorded. */
vdbc_status vdbc_batch_capture(vdbc_batch* plan, void* stream);
vdbc_status vdbc_batch_graph_launch(vdbc_batch* plan, void* stream);
void vdbc_batch_destroy(vdbc_batch* plan);

/* Philox4x32-10 (Salmon et al., SC'11) on the device: out[4i..4i+3] =
 * Philox(ctr[4i..4i+3], key[2i..2i+1]) for i < n (device uint32 arrays). */
vdbc_status vdbc_philox(const uint32_t* ctr, const uint32_t* key, uint64_t n, uint32_t* out,
                        void* stream);

/* ------------------------------------------------------------------------ */
/* Learned denoiser (this project's extension; not part of the paper)        */
/* ------------------------------------------------------------------------ */
/* A 6-layer 3x3 convolutional U-Net on NHWC tensors, BF16 weights and
 * activations, FP32 accumulation on BF16 matrix cores:
 *   c1 = relu(conv(x, 8->32)); c2 = relu(conv(c1, 32->64, stride 2));
 *   c3 = relu(conv(c2, 64->64)); c4 = relu(conv(up2(c3), 64->32));
 *   c5 = relu(conv(concat(c1, c4), 64->32)); out = x.rgb + conv(c5, 32->3).
 * x: BF16 [n][h][w][8] = (r, g, b, first-scatter depth fraction, primary
 * transmittance, 0, 0, 0) of a low-sample-count render; out: FP32 [n][h][w][3].
 * Parameters: one flat FP32 vector, per layer W[co][ky][kx][ci] then b[co];
 * `wbf16` is a BF16 copy of the whole vector (same indices).  h and w even. */
vdbc_status vdbc_nn_param_count(uint64_t* count);
/* wbf16[i] = bf16(params[i]) (round to nearest even), device arrays. */
vdbc_status vdbc_nn_to_bf16(const float* params, uint16_t* wbf16, void* stream);
/* Workspace bytes for inference (training = 0) or one training step. */
vdbc_status vdbc_denoise_workspace(uint32_t n, uint32_t h, uint32_t w, uint32_t training,
                                   uint64_t* bytes);
/* x[p] = (rgba[p].rgb, aov[p].depth, aov[p].transmittance, 0, 0, 0) as BF16,
 * from vdbc_render's image and AOV outputs (pixels = n*h*w). */
vdbc_status vdbc_denoise_pack(const float* rgba, const float* aov, uint64_t pixels, uint16_t* x,
                              void* stream);
/* Inference: out = network(x).  ws 256-byte aligned, x and wbf16 16-byte. */
vdbc_status vdbc_denoise(const float* params, const uint16_t* wbf16, const uint16_t* x, uint32_t n,
                         uint32_t h, uint32_t w, float* out, void* ws, uint64_t ws_bytes,
                         void* stream);
/* One training step on a batch: forward, loss = mean over pixels and RGB of
 * (out - t)^2 / (t^2 + 0.01) written to *loss (device float), backward, and
 * (lr > 0) one Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected with
 * `step` >= 1) on the FP32 master params with refreshed BF16 copy.  grad_out
 * (device float[param_count] or NULL) receives the gradient. */
vdbc_status vdbc_denoise_train_step(float* params, uint16_t* wbf16, float* adam_m, float* adam_v,
                                    uint32_t step, float lr, const uint16_t* x, const float* target,
                                    uint32_t n, uint32_t h, uint32_t w, float* loss,
                                    float* grad_out, void* ws, uint64_t ws_bytes, void* stream);
/* Single 3x3 convolution layer (zero padding 1): input channels [0, ca) from
 * a and [ca, ca+cb) from b (NHWC, hs x ws_, nearest x2 upsampled if
 * `upsample`), weights BF16 [cout][3][3][ca+cb], bias FP32; output BF16 or
 * FP32 (exactly one non-NULL), ReLU if `relu`.  Channels multiples of 8 up
 * to 64, cout 1..64, stride 1 or 2. */
vdbc_status vdbc_conv3x3(const uint16_t* a, uint32_t ca, const uint16_t* b, uint32_t cb,
                         uint32_t upsample, uint32_t n, uint32_t hs, uint32_t ws_, uint32_t stride,
                         const uint16_t* w, const float* bias, uint32_t cout, uint32_t relu,
                         uint16_t* out_bf16, float* out_f32, void* stream);
vdbc_status vdbc_conv3x3_grad_workspace(uint32_t cin, uint32_t cout, uint32_t n, uint32_t ho,
                                        uint32_t wo, uint64_t* bytes);
/* Data gradient: dx (FP32 [n][hv][wv][cin]) from dz (BF16 [n][ho][wo][coutp],
 * channels >= cout zero) and the layer's weights. */
vdbc_status vdbc_conv3x3_dgrad(const uint16_t* dz, uint32_t coutp, uint32_t cout, uint32_t n,
                               uint32_t ho, uint32_t wo, const uint16_t* w, uint32_t cin,
                               uint32_t stride, uint32_t hv, uint32_t wv, float* dx, void* ws,
                               uint64_t ws_bytes, void* stream);
/* Weight and bias gradients (FP32 dw[cout][3][3][cin], db[cout]) of the
 * layer whose input is described as in vdbc_conv3x3. */
vdbc_status vdbc_conv3x3_wgrad(const uint16_t* a, uint32_t ca, const uint16_t* b, uint32_t cb,
                               uint32_t upsample, uint32_t n, uint32_t hs, uint32_t ws_,
                               uint32_t stride, const uint16_t* dz, uint32_t coutp, uint32_t cout,
                               float* dw, float* db, void* ws, uint64_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif
