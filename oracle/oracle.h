/*
 * CPU oracle for compressed-VDB volume sampling and rendering.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, single-threaded
 * statement of what the GPU path computes.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it; the product path
 * never links, imports or calls it, and it shares no code, header, table or
 * helper with the product library.
 *
 * Everything follows "GPU Volume Rendering with Hierarchical Compression Using
 * VDB" (Zellmann, Jaros, Amstutz, Wald), cited by section / algorithm /
 * equation / table.  Floating point accumulates in double unless a step is
 * defined on stored float32 values (voxels, sample positions).
 *
 * Canonical buffer (format v1) written by ref_encode and walked by the lookup:
 *   header 256 B | root u32[] | upper nodes | lower nodes | upper tile f32[] |
 *   lower tile f32[] | leaf value masks u64[8] per leaf | leaf values f32[512]
 *   per leaf.  Every section starts on a 256-byte boundary.
 *   Internal node = array of 32-byte word records
 *     { u64 child_mask; u32 child_index; u32 tile_index; u64 tile_mask; u64 0 }
 *   (512 records for an upper node = 32^3 slots, 64 for a lower = 16^3 slots);
 *   child_index / tile_index are the absolute array index of the first child /
 *   tile at or after the word's first slot.  Slots, leaf voxels and the root
 *   table are x-fastest.
 */
#ifndef VDBC_ORACLE_H
#define VDBC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { REF_OK = 0, REF_E_INVALID = 1, REF_E_NOMEM = 2, REF_E_FORMAT = 4 };
enum { REF_BG_EXPLICIT = 1u, REF_NO_CORNERS = 2u, REF_NO_PRUNE = 4u, REF_PARTIAL = 8u };

typedef struct {
    float background;
    uint64_t n_bricks, k_bricks, n_leaf, n_lower, n_upper, n_lower_tiles,
        n_upper_tiles, active_voxels, bytes;
    double achieved_rate;
} ref_stats;

/* ---- Philox4x32-10 (Salmon et al., SC'11), the counter-based RNG ---- */
void ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void ref_philox_many(const uint32_t* ctr, const uint32_t* key, uint64_t n, uint32_t* out);
double ref_u01(uint32_t x);

/* ---- Alg. 1 "Compress", steps in the paper's order ---- */
/* Background: exact mode of the float values (-0 counted as +0, ties to the
 * smallest value).  Alg. 1 histogram/argmax; Section 3.1 phase 1. */
float ref_background(const float* dense, uint64_t n);
/* Brick value ranges over 32^3 bricks (partial edge bricks included). */
void ref_brick_ranges(const float* dense, uint32_t nx, uint32_t ny, uint32_t nz,
                      float* lo, float* hi);
/* Similarity of a brick range to B, Eq. (1)-(3); metric 1 closest, 2 farthest,
 * 3 median point-in-range. */
double ref_similarity(uint32_t metric, float lo, float hi, float B);
/* Sorted brick order (most dissimilar first, ties by brick index) and K. */
int ref_brick_order(const float* dense, uint32_t nx, uint32_t ny, uint32_t nz,
                    float rate, uint32_t metric, float B, uint32_t* order,
                    uint64_t* k_out);
/* Reconstructed grid R: original value where the voxel was activated, B
 * elsewhere (decode-to-dense computed from the selection, not the buffer). */
int ref_reconstruct(const float* dense, uint32_t nx, uint32_t ny, uint32_t nz,
                    float rate, uint32_t metric, uint32_t flags, float bg,
                    float* R);
/* Full encoder: canonical buffer, malloc'ed; free with ref_free. */
int ref_encode(const float* dense, uint32_t nx, uint32_t ny, uint32_t nz,
               float rate, uint32_t metric, uint32_t flags, float bg,
               uint8_t** out, uint64_t* bytes, ref_stats* st);
/* Partial-brick activation (Section 3.2.1 names it as future work; the rule
 * is stated in encode.c): flags must include REF_PARTIAL, pfrac in (0, 1] is
 * the share of a brick's voxels activated first, ptau the similarity from
 * which down bricks are activated partially.  The header records pfrac and
 * ptau at bytes 160 and 164. */
int ref_reconstruct_partial(const float* dense, uint32_t nx, uint32_t ny, uint32_t nz,
                            float rate, uint32_t metric, uint32_t flags, float bg, float pfrac,
                            float ptau, float* R);
int ref_encode_partial(const float* dense, uint32_t nx, uint32_t ny, uint32_t nz,
                       float rate, uint32_t metric, uint32_t flags, float bg, float pfrac,
                       float ptau, uint8_t** out, uint64_t* bytes, ref_stats* st);
/* The activation itself: mask[i] = 1 where voxel i is active (any flags). */
int ref_active_mask(const float* dense, uint32_t nx, uint32_t ny, uint32_t nz, float rate,
                    uint32_t metric, uint32_t flags, float bg, float pfrac, float ptau,
                    uint8_t* mask);
void ref_free(void* p);

/* ---- Field access (Section 3.2.2): lookup, nearest, trilinear ---- */
typedef struct {
    int kind;                 /* 0 = canonical VDB buffer, 1 = dense array */
    const uint8_t* buf;       /* kind 0 */
    uint64_t bytes;
    const float* dense;       /* kind 1, x-fastest */
    uint32_t nx, ny, nz;
    float background;
} ref_field;

int ref_field_vdb(ref_field* f, const uint8_t* buf, uint64_t bytes);
void ref_field_dense(ref_field* f, const float* dense, uint32_t nx, uint32_t ny,
                     uint32_t nz, float background);
float ref_lookup(const ref_field* f, int64_t i, int64_t j, int64_t k);
void ref_lookup_many(const ref_field* f, const int64_t* ijk, uint64_t n, float* out);
double ref_sample(const ref_field* f, const float p[3], uint32_t filter);
void ref_sample_many(const ref_field* f, const float* pos, uint64_t n,
                     uint32_t filter, double* out);

/* ---- Rendering (Section 4) ---- */
typedef struct {
    uint32_t kind;            /* 0 orthographic, 1 pinhole */
    uint32_t width, height;
    float origin[3];          /* pinhole eye; unused for orthographic */
    float lower_left[3];      /* pinhole: direction to pixel (0,0) corner;
                                 ortho: ray origin of pixel (0,0) corner */
    float du[3], dv[3];       /* per-pixel steps */
    float dir[3];             /* ortho ray direction */
} ref_camera;

typedef struct {
    float sigma_scale;        /* extinction per unit of the longest axis at alpha=1 */
    float albedo;
    uint32_t tf_n;            /* 2..64 RGBA control points over [tf_lo, tf_hi] */
    float tf[64][4];
    float tf_lo, tf_hi;
    float light_dir[3];       /* unit vector pointing towards the light */
    float light_E[3];
    float ambient[3];
    const float* env;         /* NULL or [env_h][env_w][3] lat-long radiance seen by
                                 escaping path-tracer rays instead of ambient (R25) */
    uint32_t env_w, env_h;
} ref_medium;

typedef struct {
    uint32_t spp, max_bounces, macrocell;
    float step;               /* EA step in voxels */
    float t_terminate;        /* EA early termination threshold, 0 = off */
    uint64_t seed;
    uint32_t frame;
    uint32_t rr;              /* path tracer: Russian roulette (reading R24) */
} ref_render_params;

/* Majorant grid (Section 4, macrocells): per cell the extinction max over the
 * one-voxel-dilated footprint.  Grid ceil(n/C) per axis, x-fastest. */
int ref_majorant(const ref_field* f, const ref_medium* m, uint32_t C, double* maj);
/* The majorant of the cells with flat index (x-fastest) in [begin, end)
 * only; ref_majorant is [0, cells). */
int ref_majorant_cells(const ref_field* f, const ref_medium* m, uint32_t C, uint64_t begin,
                       uint64_t end, double* maj);
/* Emission-absorption ray marching; image RGBA double [h][w][4]. */
int ref_render_ea(const ref_field* f, const ref_camera* c, const ref_medium* m,
                  const ref_render_params* r, double* image);
/* Delta-tracking path tracer, for a list of pixel indices (py*W+px).
 * rgba[n][4] = mean radiance and mean primary opacity; aov[n][2] (may be
 * NULL) = mean first-scatter depth fraction and primary transmittance. */
int ref_render_pt(const ref_field* f, const ref_camera* c, const ref_medium* m,
                  const ref_render_params* r, const uint32_t* pixels,
                  uint64_t n_pixels, double* rgba, double* aov);
/* ref_render_pt over a majorant grid the caller computed with ref_majorant
 * (or ref_majorant_cells over every cell) at r->macrocell. */
int ref_render_pt_majorant(const ref_field* f, const ref_camera* c, const ref_medium* m,
                           const ref_render_params* r, const double* maj, const uint32_t* pixels,
                           uint64_t n_pixels, double* rgba, double* aov);
/* Implicit iso-surface ray marcher (the interval-based marcher of Section
 * 5.4, reading R22): one ray per pixel centre, field samples at
 * t0 + (k + 1/2) step; the first interval between consecutive samples whose
 * sides of the iso value differ (side = f >= iso) is refined by `refine`
 * bisection steps; the hit is the midpoint of the final interval; the normal
 * is -grad f / |grad f| with central differences of half a voxel.
 * image[h][w][4] = (0.5 (n + 1), 1) on a hit, 0 otherwise.  aux[h][w][3]
 * (may be NULL) = (ray parameter of the hit or -1, min |f - iso| over the
 * lattice samples up to the hit (all of them on a miss), min |f - iso| over
 * the bisection midpoints (+inf if none)). */
int ref_render_iso(const ref_field* f, const ref_camera* c, double iso, double step,
                   uint32_t refine, double* image, double* aux);
/* Uniform direction on the sphere from two uniforms (isotropic phase). */
void ref_isotropic(double u1, double u2, double d[3]);
/* Mean of `trials` binary delta-tracking transmittance estimates along one
 * ray (origin o, unit direction d) through the whole box (pins free flight). */
double ref_transmittance(const ref_field* f, const ref_medium* m, uint32_t C,
                         const float o[3], const float d[3], uint64_t trials,
                         uint64_t seed);

#ifdef __cplusplus
}
#endif
#endif
