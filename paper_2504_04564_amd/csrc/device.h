// Device-side building blocks for gfx950: Philox4x32-10, the VDB and dense
// field accessors, trilinear reconstruction, transfer function, camera rays.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "format.h"

namespace vdbc {

// ---------------------------------------------------------------- Philox
// Philox4x32-10 from its published definition (Salmon et al., SC'11, Section
// 4): S-box multipliers 0xD2511F53 / 0xCD9E8D57, Weyl key increments
// 0x9E3779B9 / 0xBB67AE85, ten rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                              uint32_t& c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // one 32 x 32 -> 64-bit product per multiplier (a single
        // v_mad_u64_u32 instead of separate high- and low-half multiplies)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
    }
}

// One random stream of a path: key (seed_lo ^ pixel, seed_hi), counter
// (block, sample, stream << 16 | bounce, frame); draw d is word d & 3 of
// block d >> 2; u = (x >> 8) * 2^-24.
struct Rng {
    uint32_t k0, k1, sample, tag, frame;
    uint32_t d;
    uint32_t w0, w1, w2, w3;

    __device__ void init(uint32_t key0, uint32_t key1, uint32_t s, uint32_t bounce,
                         uint32_t stream, uint32_t f)
    {
        k0 = key0;
        k1 = key1;
        sample = s;
        tag = (stream << 16) | bounce;
        frame = f;
        d = 0;
    }
    __device__ __forceinline__ float next()
    {
        const uint32_t q = d & 3u;
        if (q == 0) {
            w0 = d >> 2;
            w1 = sample;
            w2 = tag;
            w3 = frame;
            philox4x32_10(w0, w1, w2, w3, k0, k1);
        }
        ++d;
        const uint32_t x = q == 0 ? w0 : q == 1 ? w1 : q == 2 ? w2 : w3;
        return (float)(x >> 8) * (1.0f / 16777216.0f);
    }
};

// ---------------------------------------------------------------- fields

// Where the 512 values of a leaf-sized region live: value(n3) = p[n3 & m].
// A stored leaf has m = 511; a tile or an empty region points at one float
// (the tile value, or the background in the buffer header) with m = 0, so
// every corner fetch is a plain load without branches.
struct LeafH {
    const float* p;
    uint32_t m;
};

struct VdbView {
    const uint32_t* root;
    const Word* upper;
    const Word* lower;
    const float* upper_tiles;
    const float* lower_tiles;
    const float* leaf_values;
    const float* bg;   // background value inside the header
    int nx, ny, nz;
    int rnx, rny, rnz;
    float background;
};

__device__ __forceinline__ uint32_t popc64(uint64_t x) { return __popcll(x); }
__device__ __forceinline__ uint64_t below(uint32_t bit) { return (uint64_t(1) << bit) - 1u; }

// What a VDB accessor keeps between consecutive lookups of one thread: nothing
// (every lookup descends from the root), the last leaf region, or the last
// leaf region and the last lower node.  The policy changes only the work of a
// lookup, never its value.
enum CachePolicy { kCacheNone = 0, kCacheLeaf = 1, kCacheLeafLower = 2 };

// Random-access VDB accessor with a per-thread cache (policy CP) of the last
// lower node and the last leaf, reused across consecutive samples of one thread.
template <int CP>
struct VdbAccT {
    static constexpr bool kTree = true;   // regions resolvable leaf by leaf
    VdbView v;
    int clx, cly, clz;       // cached leaf coordinates (voxel >> 3)
    LeafH cleaf;
    int cLx, cLy, cLz;       // cached lower-node coordinates (voxel >> 7)
    const Word* cnode;       // cached lower node, or null for a constant region
    const float* cconst;

    __device__ void reset()
    {
        clx = cly = clz = 0x40000000;
        cLx = cLy = cLz = 0x40000000;
        cnode = nullptr;
        cconst = v.bg;
        cleaf = LeafH{v.bg, 0};
    }

    __device__ __forceinline__ float background() const { return v.background; }

    __device__ void resolve_lower(int Lx, int Ly, int Lz)
    {
        cLx = Lx;
        cLy = Ly;
        cLz = Lz;
        cnode = nullptr;
        cconst = v.bg;
        const int Ux = Lx >> 5, Uy = Ly >> 5, Uz = Lz >> 5;
        if (Ux >= v.rnx || Uy >= v.rny || Uz >= v.rnz) return;
        const uint32_t u = v.root[Ux + v.rnx * (Uy + v.rny * Uz)];
        if (u == kNoChild) return;
        const uint32_t n1 = (Lx & 31) + 32u * ((Ly & 31) + 32u * (Lz & 31));
        const Word* w = v.upper + (uint64_t)u * kUpperWords + (n1 >> 6);
        const uint32_t bit = n1 & 63u;
        const uint64_t child = w->child;
        if ((child >> bit) & 1u) {
            cnode = v.lower + (uint64_t)(w->child_index + popc64(child & below(bit))) * kLowerWords;
            return;
        }
        const uint64_t tile = w->tile;
        if ((tile >> bit) & 1u) cconst = v.upper_tiles + w->tile_index + popc64(tile & below(bit));
    }

    // Region of leaf (lx,ly,lz); negative coordinates and regions without a
    // voxel read the background.
    __device__ LeafH resolve(int lx, int ly, int lz)
    {
        if (CP >= kCacheLeaf && lx == clx && ly == cly && lz == clz) return cleaf;
        LeafH h{v.bg, 0};
        if ((lx | ly | lz) >= 0) {
            const int Lx = lx >> 4, Ly = ly >> 4, Lz = lz >> 4;
            if (CP < kCacheLeafLower || Lx != cLx || Ly != cLy || Lz != cLz) resolve_lower(Lx, Ly, Lz);
            if (!cnode) {
                h.p = cconst;
            } else {
                const uint32_t n2 = (lx & 15) + 16u * ((ly & 15) + 16u * (lz & 15));
                const Word* w = cnode + (n2 >> 6);
                const uint32_t bit = n2 & 63u;
                const uint64_t child = w->child;
                if ((child >> bit) & 1u) {
                    h.p = v.leaf_values +
                          (uint64_t)(w->child_index + popc64(child & below(bit))) * kLeafVoxels;
                    h.m = 511u;
                } else {
                    const uint64_t tile = w->tile;
                    if ((tile >> bit) & 1u)
                        h.p = v.lower_tiles + w->tile_index + popc64(tile & below(bit));
                }
            }
        }
        if (CP >= kCacheLeaf) {
            clx = lx;
            cly = ly;
            clz = lz;
            cleaf = h;
        }
        return h;
    }

    __device__ __forceinline__ float voxel(int i, int j, int k)
    {
        const LeafH h = resolve(i >> 3, j >> 3, k >> 3);
        return h.p[((i & 7) + 8 * (j & 7) + 64 * (k & 7)) & h.m];
    }

    // The eight corners of the cell with lower corner (i,j,k), x fastest.
    __device__ __forceinline__ void corners(int i, int j, int k, float c[8])
    {
        const int lx0 = i >> 3, ly0 = j >> 3, lz0 = k >> 3;
        const bool sx = (i & 7) == 7, sy = (j & 7) == 7, sz = (k & 7) == 7;
        const uint32_t a0 = (i & 7) + 8 * (j & 7) + 64 * (k & 7);
        const uint32_t ax = sx ? a0 - 7 : a0 + 1;       // x+1 within its leaf
        const uint32_t ay = sy ? -56u : 8u;              // y step
        const uint32_t az = sz ? -448u : 64u;            // z step
        // One code path for every footprint: a footprint inside one leaf takes
        // h000 for all corners through the selects below.  A separate early
        // return for that case costs more than it saves, since nearly every
        // wave holds lanes of both kinds and would run both load sequences.
        const LeafH h000 = resolve(lx0, ly0, lz0);
        const LeafH h100 = sx ? resolve(lx0 + 1, ly0, lz0) : h000;
        const LeafH h010 = sy ? resolve(lx0, ly0 + 1, lz0) : h000;
        const LeafH h110 = sy ? (sx ? resolve(lx0 + 1, ly0 + 1, lz0) : h010) : h100;
        const LeafH h001 = sz ? resolve(lx0, ly0, lz0 + 1) : h000;
        const LeafH h101 = sz ? (sx ? resolve(lx0 + 1, ly0, lz0 + 1) : h001) : h100;
        const LeafH h011 = sz ? (sy ? resolve(lx0, ly0 + 1, lz0 + 1) : h001) : h010;
        const LeafH h111 =
            sz ? (sy ? (sx ? resolve(lx0 + 1, ly0 + 1, lz0 + 1) : h011) : h101) : h110;
        const uint32_t b0 = a0, b1 = ax;
        c[0] = h000.p[b0 & h000.m];
        c[1] = h100.p[b1 & h100.m];
        c[2] = h010.p[(b0 + ay) & h010.m];
        c[3] = h110.p[(b1 + ay) & h110.m];
        c[4] = h001.p[(b0 + az) & h001.m];
        c[5] = h101.p[(b1 + az) & h101.m];
        c[6] = h011.p[(b0 + ay + az) & h011.m];
        c[7] = h111.p[(b1 + ay + az) & h111.m];
    }

    // log2 edge of the largest empty aligned node region (no child, no tile)
    // holding voxel (i,j,k): 12 (no upper node), 7 (empty lower slot),
    // 3 (empty leaf slot), 0 (a leaf or tile is there, or i,j,k < 0).
    // True when voxel (i,j,k) lies in the cached leaf and that leaf stores
    // voxels: the sample is then not inside an empty node (no query needed).
    __device__ __forceinline__ bool in_stored_leaf(int i, int j, int k) const
    {
        return CP >= kCacheLeaf && (i >> 3) == clx && (j >> 3) == cly && (k >> 3) == clz && cleaf.m != 0u;
    }

    __device__ int empty_level(int i, int j, int k)
    {
        if ((i | j | k) < 0) return 0;
        const int lx = i >> 3, ly = j >> 3, lz = k >> 3;
        const int Lx = lx >> 4, Ly = ly >> 4, Lz = lz >> 4;
        if (CP < kCacheLeafLower || Lx != cLx || Ly != cLy || Lz != cLz) resolve_lower(Lx, Ly, Lz);
        if (!cnode) {
            if (cconst != v.bg) return 0;                 // an upper tile
            const int Ux = Lx >> 5, Uy = Ly >> 5, Uz = Lz >> 5;
            if (Ux >= v.rnx || Uy >= v.rny || Uz >= v.rnz) return 12;
            return v.root[Ux + v.rnx * (Uy + v.rny * Uz)] == kNoChild ? 12 : 7;
        }
        const uint32_t n2 = (lx & 15) + 16u * ((ly & 15) + 16u * (lz & 15));
        const Word* w = cnode + (n2 >> 6);
        const uint32_t bit = n2 & 63u;
        return (((w->child | w->tile) >> bit) & 1u) ? 0 : 3;
    }
};

using VdbAcc = VdbAccT<kCacheLeafLower>;

struct DenseView {
    const float* data;
    int nx, ny, nz;
    float background;
};

// The "3D texture" baseline: a plain x-fastest float32 array read in
// software, background outside the volume.
struct DenseAcc {
    static constexpr bool kTree = false;
    DenseView v;
    __device__ void reset() {}
    __device__ __forceinline__ float background() const { return v.background; }
    __device__ __forceinline__ float voxel(int i, int j, int k)
    {
        const bool in = (unsigned)i < (unsigned)v.nx && (unsigned)j < (unsigned)v.ny &&
                        (unsigned)k < (unsigned)v.nz;
        const int ci = in ? i : 0, cj = in ? j : 0, ck = in ? k : 0;
        const float x = v.data[ci + (int64_t)v.nx * (cj + (int64_t)v.ny * ck)];
        return in ? x : v.background;
    }
    __device__ __forceinline__ void corners(int i, int j, int k, float c[8])
    {
        const bool ix0 = (unsigned)i < (unsigned)v.nx, ix1 = (unsigned)(i + 1) < (unsigned)v.nx;
        const bool iy0 = (unsigned)j < (unsigned)v.ny, iy1 = (unsigned)(j + 1) < (unsigned)v.ny;
        const bool iz0 = (unsigned)k < (unsigned)v.nz, iz1 = (unsigned)(k + 1) < (unsigned)v.nz;
        const int x0 = ix0 ? i : 0, x1 = ix1 ? i + 1 : 0;
        const int64_t sy = v.nx, sz = (int64_t)v.nx * v.ny;
        const int64_t y0 = (iy0 ? j : 0) * sy, y1 = (iy1 ? j + 1 : 0) * sy;
        const int64_t z0 = (iz0 ? k : 0) * sz, z1 = (iz1 ? k + 1 : 0) * sz;
        const float* d = v.data;
        const float B = v.background;
        c[0] = (ix0 & iy0 & iz0) ? d[x0 + y0 + z0] : B;
        c[1] = (ix1 & iy0 & iz0) ? d[x1 + y0 + z0] : B;
        c[2] = (ix0 & iy1 & iz0) ? d[x0 + y1 + z0] : B;
        c[3] = (ix1 & iy1 & iz0) ? d[x1 + y1 + z0] : B;
        c[4] = (ix0 & iy0 & iz1) ? d[x0 + y0 + z1] : B;
        c[5] = (ix1 & iy0 & iz1) ? d[x1 + y0 + z1] : B;
        c[6] = (ix0 & iy1 & iz1) ? d[x0 + y1 + z1] : B;
        c[7] = (ix1 & iy1 & iz1) ? d[x1 + y1 + z1] : B;
    }
    __device__ bool in_stored_leaf(int, int, int) const { return true; }
    __device__ int empty_level(int, int, int) { return 0; }
};

// ---------------------------------------------------------------- sampling

__device__ __forceinline__ float lerp(float a, float b, float t) { return fmaf(t, b - a, a); }

// Positions far outside the volume are clamped first (every corner there
// reads B and lerp(B, B, t) == B, so the value is unchanged) so that the
// float -> int conversion stays in range.
template <class Acc>
__device__ __forceinline__ float trilinear(Acc& acc, float px, float py, float pz)
{
    px = fminf(fmaxf(px, -2.0f), (float)acc.v.nx + 1.0f);
    py = fminf(fmaxf(py, -2.0f), (float)acc.v.ny + 1.0f);
    pz = fminf(fmaxf(pz, -2.0f), (float)acc.v.nz + 1.0f);
    const float fx0 = floorf(px), fy0 = floorf(py), fz0 = floorf(pz);
    const float fx = px - fx0, fy = py - fy0, fz = pz - fz0;
    float c[8];
    acc.corners((int)fx0, (int)fy0, (int)fz0, c);
    const float c00 = lerp(c[0], c[1], fx), c10 = lerp(c[2], c[3], fx);
    const float c01 = lerp(c[4], c[5], fx), c11 = lerp(c[6], c[7], fx);
    return lerp(lerp(c00, c10, fy), lerp(c01, c11, fy), fz);
}

template <class Acc>
__device__ __forceinline__ float nearest(Acc& acc, float px, float py, float pz)
{
    px = fminf(fmaxf(px, -2.0f), (float)acc.v.nx + 1.0f);
    py = fminf(fmaxf(py, -2.0f), (float)acc.v.ny + 1.0f);
    pz = fminf(fmaxf(pz, -2.0f), (float)acc.v.nz + 1.0f);
    const float fx0 = floorf(px), fy0 = floorf(py), fz0 = floorf(pz);
    const int i = (int)fx0 + ((px - fx0) >= 0.5f);
    const int j = (int)fy0 + ((py - fy0) >= 0.5f);
    const int k = (int)fz0 + ((pz - fz0) >= 0.5f);
    return acc.voxel(i, j, k);
}

// ---------------------------------------------------------------- medium

struct MediumK {
    float ds;          // sigma_scale / max(n): extinction per voxel at alpha = 1
    float albedo;
    int tf_n;
    float tf_lo, tf_inv;  // (tf_n - 1) / (tf_hi - tf_lo)
    float4 tf[64];
    float light[3], light_E[3], ambient[3];
    const float* env;  // lat-long escape radiance [env_h][env_w][3], or null
    int env_w, env_h;
};

// Radiance seen by a ray leaving the volume along unit direction d: the
// constant ambient, or the nearest texel of the lat-long map at
// u = (atan2(d_z, d_x) + pi) / 2 pi, v = acos(d_y) / pi.
__device__ __forceinline__ void escape_radiance(const MediumK& m, const float d[3], float& r, float& g,
                                                float& b)
{
    if (!m.env) {
        r = m.ambient[0];
        g = m.ambient[1];
        b = m.ambient[2];
        return;
    }
    const float u = (atan2f(d[2], d[0]) + 3.14159265358979323846f) * 0.159154943091895335769f;
    const float v = acosf(fminf(fmaxf(d[1], -1.0f), 1.0f)) * 0.318309886183790671538f;
    const int tx = min(max((int)floorf(u * (float)m.env_w), 0), m.env_w - 1);
    const int ty = min(max((int)floorf(v * (float)m.env_h), 0), m.env_h - 1);
    const float* p = m.env + 3 * ((size_t)ty * (size_t)m.env_w + (size_t)tx);
    r = p[0];
    g = p[1];
    b = p[2];
}

__device__ __forceinline__ float4 tf_eval(const MediumK& m, float s)
{
    float pos = (s - m.tf_lo) * m.tf_inv;
    pos = fminf(fmaxf(pos, 0.0f), (float)(m.tf_n - 1));
    int i = (int)pos;
    i = i > m.tf_n - 2 ? m.tf_n - 2 : i;
    const float fr = pos - (float)i;
    const float4 a = m.tf[i], b = m.tf[i + 1];
    return make_float4(lerp(a.x, b.x, fr), lerp(a.y, b.y, fr), lerp(a.z, b.z, fr),
                       lerp(a.w, b.w, fr));
}

// tf_alpha with the control points read from `tf` (an LDS copy of m.tf).
__device__ __forceinline__ float tf_alpha_at(const float4* tf, const MediumK& m, float s)
{
    float pos = (s - m.tf_lo) * m.tf_inv;
    pos = fminf(fmaxf(pos, 0.0f), (float)(m.tf_n - 1));
    int i = (int)pos;
    i = i > m.tf_n - 2 ? m.tf_n - 2 : i;
    const float fr = pos - (float)i;
    return lerp(tf[i].w, tf[i + 1].w, fr);
}

__device__ __forceinline__ float tf_alpha(const MediumK& m, float s)
{
    float pos = (s - m.tf_lo) * m.tf_inv;
    pos = fminf(fmaxf(pos, 0.0f), (float)(m.tf_n - 1));
    int i = (int)pos;
    i = i > m.tf_n - 2 ? m.tf_n - 2 : i;
    const float fr = pos - (float)i;
    return lerp(m.tf[i].w, m.tf[i + 1].w, fr);
}

// ---------------------------------------------------------------- camera

struct CameraK {
    int kind, width, height;
    float o[3], ll[3], du[3], dv[3], dir[3];
};

__device__ __forceinline__ void camera_ray(const CameraK& c, float x, float y, float o[3],
                                           float d[3])
{
    float len2 = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float t = fmaf(x, c.du[a], fmaf(y, c.dv[a], c.ll[a]));
        if (c.kind == 1) {
            o[a] = c.o[a];
            d[a] = t;
        } else {
            o[a] = t;
            d[a] = c.dir[a];
        }
        len2 = fmaf(d[a], d[a], len2);
    }
    const float inv = 1.0f / sqrtf(len2);
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] *= inv;
}

// Ray / box [-0.5, n-0.5]^3 with the direction's reciprocals id = 1/d;
// t0 clamped to >= 0.
__device__ __forceinline__ bool box_clip(int nx, int ny, int nz, const float o[3],
                                         const float d[3], const float id[3], float& t0, float& t1)
{
    const float hi[3] = {(float)nx - 0.5f, (float)ny - 0.5f, (float)nz - 0.5f};
    float lo_t = -INFINITY, hi_t = INFINITY;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0f) {
            if (o[a] < -0.5f || o[a] > hi[a]) return false;
            continue;
        }
        const float ta = (-0.5f - o[a]) * id[a], tb = (hi[a] - o[a]) * id[a];
        lo_t = fmaxf(lo_t, fminf(ta, tb));
        hi_t = fminf(hi_t, fmaxf(ta, tb));
    }
    t0 = fmaxf(lo_t, 0.0f);
    t1 = hi_t;
    // a zero or non-finite direction leaves t1 infinite: no segment
    return t0 < t1 && t1 <= 1.0e30f;
}

}  // namespace vdbc
