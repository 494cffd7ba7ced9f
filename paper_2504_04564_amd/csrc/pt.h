// Device code of the delta-tracking path tracer (Section 4): majorant-grid
// DDA with coarse-block skipping, the per-tile path pool, the persistent
// single-volume kernel and the batched multi-volume kernel.
#pragma once
#include "kcommon.h"

namespace vdbc {

// Resident PT workgroups per compute unit (the kernel's launch bounds).
constexpr int kPtBlocksPerCu = 4;
// Largest samples per pixel (256 x spp work units per tile fit 32 bits) and
// bounces per path (the bounce is a 16-bit field of the Philox counter).
constexpr uint32_t kMaxSpp = 1u << 16;
constexpr uint32_t kMaxBounces = 0xFFFFu;

// ---------------------------------------------------------------- PT

struct PtArgs {
    int spp, max_bounces, C, gx, gy, gz, tw;
    float invC;
    int lf, cgx, cgy, cgz, cwords;   // coarse blocks of 2^lf macrocells per axis, bit words
    uint32_t seed_lo, seed_hi, frame;
    int rr;                          // Russian roulette from bounce 2 on
    uint32_t chunk, chunks;          // samples per work item, work items per tile
};

// Occupancy of the coarse blocks: bit set iff some macrocell of the block has
// a non-zero majorant.  One thread per block; a wave ballot assembles two
// 32-bit words per wave.
// Workgroup `blk` of that launch (the whole workgroup calls it).
__device__ inline void coarse_bits_block(const float* __restrict__ maj, const PtArgs& g, uint32_t* __restrict__ bits,
                                         uint32_t blk)
{
    const int cell = (int)blk * blockDim.x + threadIdx.x;
    const int ncoarse = g.cgx * g.cgy * g.cgz;
    const int F = 1 << g.lf;
    bool occ = false;
    if (cell < ncoarse) {
        const int bx = cell % g.cgx, by = (cell / g.cgx) % g.cgy, bz = cell / (g.cgx * g.cgy);
        for (int z = bz * F; z < min(bz * F + F, g.gz) && !occ; ++z)
            for (int y = by * F; y < min(by * F + F, g.gy) && !occ; ++y)
                for (int x = bx * F; x < min(bx * F + F, g.gx); ++x)
                    if (maj[x + g.gx * (y + g.gy * z)] > 0.0f) {
                        occ = true;
                        break;
                    }
    }
    const uint64_t ballot = __ballot(occ);
    const int lane = threadIdx.x & 63;
    const int w = ((int)blk * blockDim.x + threadIdx.x - lane) >> 5;   // first word of the wave
    if (lane == 0 && w < g.cwords) bits[w] = (uint32_t)ballot;
    if (lane == 0 && w + 1 < g.cwords) bits[w + 1] = (uint32_t)(ballot >> 32);
}

__global__ __launch_bounds__(kBlock) void coarse_bits_kernel(const float* __restrict__ maj,
                                                             PtArgs g, uint32_t* __restrict__ bits)
{
    coarse_bits_block(maj, g, bits, blockIdx.x);
}

// One ray segment being tracked through the majorant grid (Section 4): a 3D
// DDA over macrocells, hierarchical over coarse blocks of macrocells whose
// occupancy bits live in LDS, and delta tracking inside non-empty cells.
struct Flight {
    float o[3], d[3], id[3];
    float t, t1, te, mu, imu;
    int cx, cy, cz, axis;
    bool incell, ok;
    uint32_t budget;
};

// Starts a segment: clip to the box and find the first macrocell.
__device__ __forceinline__ void flight_begin(Flight& f, const PtArgs& g, int nx, int ny, int nz,
                                             const float o[3], const float d[3], float& t0)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        f.o[a] = o[a];
        f.d[a] = d[a];
        f.id[a] = __builtin_amdgcn_rcpf(d[a]);   // hardware reciprocal (<= 1 ulp; 1/0 -> inf)
    }
    f.incell = false;
    f.budget = kMaxFlightSamples;
    f.ok = box_clip(nx, ny, nz, o, d, f.id, t0, f.t1);
    f.t = t0;
    if (!f.ok) return;
    // the macrocell edge is a power of two: multiplying by its reciprocal is exact
    f.cx = min(max((int)floorf((fmaf(t0, d[0], o[0]) + 0.5f) * g.invC), 0), g.gx - 1);
    f.cy = min(max((int)floorf((fmaf(t0, d[1], o[1]) + 0.5f) * g.invC), 0), g.gy - 1);
    f.cz = min(max((int)floorf((fmaf(t0, d[2], o[2]) + 0.5f) * g.invC), 0), g.gz - 1);
}

__device__ __forceinline__ bool coarse_occupied(const uint32_t* bits, const PtArgs& g, int bx,
                                                int by, int bz)
{
    const uint32_t i = (uint32_t)(bx + g.cgx * (by + g.cgy * bz));
    return (bits[i >> 5] >> (i & 31u)) & 1u;
}

// Exit distance through the faces of an axis-aligned cell of edge `edge`
// (index c along each axis); returns the crossing axis or -1 if t1 is closer.
__device__ __forceinline__ int cell_exit(const Flight& f, float edge, int cx, int cy, int cz,
                                         float& te)
{
    te = f.t1;
    int axis = -1;
    if (f.d[0] != 0.0f) {
        const float ta = (edge * (float)(cx + (f.d[0] > 0.0f)) - 0.5f - f.o[0]) * f.id[0];
        if (ta < te) {
            te = ta;
            axis = 0;
        }
    }
    if (f.d[1] != 0.0f) {
        const float ta = (edge * (float)(cy + (f.d[1] > 0.0f)) - 0.5f - f.o[1]) * f.id[1];
        if (ta < te) {
            te = ta;
            axis = 1;
        }
    }
    if (f.d[2] != 0.0f) {
        const float ta = (edge * (float)(cz + (f.d[2] > 0.0f)) - 0.5f - f.o[2]) * f.id[2];
        if (ta < te) {
            te = ta;
            axis = 2;
        }
    }
    return axis;
}

// Advances the flight to its next tentative collision: returns 1 with f.t
// at the collision (the caller samples the density there and makes the
// accept test), 0 when the segment leaves the grid without one, or
// kFlightYield after entering kWalkCells macrocells without a collision (call
// again to continue; the walk and its random draws are the same as without
// the pause).  Empty cells draw no random
// numbers and coarse-block faces are macrocell faces, so the tentative
// collisions are those of a uniform walk over every macrocell; a flight that
// overshoots a cell restarts at its exit (memorylessness).
__device__ __forceinline__ int flight_advance(Flight& f, const float* __restrict__ maj, const uint32_t* cbits,
                                              const PtArgs& g, Rng& rng, uint32_t& ncell)
{
    if (!f.ok) return 0;
    const float C = (float)g.C;
    const float CF = (float)(g.C << g.lf);
    int walk = kWalkCells;
    for (;;) {
        if (f.incell) {
            f.t = fmaf(-__logf(1.0f - rng.next()), f.imu, f.t);
            if (f.t < f.te) {
                if (--f.budget == 0) return 0;
                return 1;
            }
            f.incell = false;
            if (f.axis < 0) return 0;
            f.t = f.te;
            if (f.axis == 0) {
                f.cx += f.d[0] > 0.0f ? 1 : -1;
                if ((unsigned)f.cx >= (unsigned)g.gx) return 0;
            } else if (f.axis == 1) {
                f.cy += f.d[1] > 0.0f ? 1 : -1;
                if ((unsigned)f.cy >= (unsigned)g.gy) return 0;
            } else {
                f.cz += f.d[2] > 0.0f ? 1 : -1;
                if ((unsigned)f.cz >= (unsigned)g.gz) return 0;
            }
        }
        if (--walk < 0) return kFlightYield;
        const int bx = f.cx >> g.lf, by = f.cy >> g.lf, bz = f.cz >> g.lf;
        ++ncell;
        if (!coarse_occupied(cbits, g, bx, by, bz)) {
            // cross the empty block in one step
            float te;
            const int axis = cell_exit(f, CF, bx, by, bz, te);
            if (axis < 0) return 0;
            f.t = te;
            const int F = 1 << g.lf;
            const float px = (fmaf(te, f.d[0], f.o[0]) + 0.5f) * g.invC;
            const float py = (fmaf(te, f.d[1], f.o[1]) + 0.5f) * g.invC;
            const float pz = (fmaf(te, f.d[2], f.o[2]) + 0.5f) * g.invC;
            if (axis == 0) {
                f.cx = f.d[0] > 0.0f ? (bx + 1) * F : bx * F - 1;
                if ((unsigned)f.cx >= (unsigned)g.gx) return 0;
            } else {
                f.cx = min(max((int)floorf(px), bx * F), min(bx * F + F, g.gx) - 1);
            }
            if (axis == 1) {
                f.cy = f.d[1] > 0.0f ? (by + 1) * F : by * F - 1;
                if ((unsigned)f.cy >= (unsigned)g.gy) return 0;
            } else {
                f.cy = min(max((int)floorf(py), by * F), min(by * F + F, g.gy) - 1);
            }
            if (axis == 2) {
                f.cz = f.d[2] > 0.0f ? (bz + 1) * F : bz * F - 1;
                if ((unsigned)f.cz >= (unsigned)g.gz) return 0;
            } else {
                f.cz = min(max((int)floorf(pz), bz * F), min(bz * F + F, g.gz) - 1);
            }
            continue;
        }
        f.axis = cell_exit(f, C, f.cx, f.cy, f.cz, f.te);
        f.mu = maj[f.cx + g.gx * (f.cy + g.gy * f.cz)];
        if (f.mu > 0.0f && f.t < f.te) {
            f.incell = true;
            f.imu = __builtin_amdgcn_rcpf(f.mu);   // hardware reciprocal (<= 1 ulp)
            continue;
        }
        if (f.axis < 0) return 0;
        f.t = f.te;
        if (f.axis == 0) {
            f.cx += f.d[0] > 0.0f ? 1 : -1;
            if ((unsigned)f.cx >= (unsigned)g.gx) return 0;
        } else if (f.axis == 1) {
            f.cy += f.d[1] > 0.0f ? 1 : -1;
            if ((unsigned)f.cy >= (unsigned)g.gy) return 0;
        } else {
            f.cz += f.d[2] > 0.0f ? 1 : -1;
            if ((unsigned)f.cz >= (unsigned)g.gz) return 0;
        }
    }
}

// LDS state of one 256-pixel tile: next unit of work and per-pixel sums in
// 2^-32 fixed point (integer sums do not depend on the order of the adds).
// Per-pixel fixed-point sums of a launch whose tiles are split into several
// work items: rgbn[4 pix + k] = red, green, blue (k < 3) and hits | escapes
// << 32 (k = 3); depth[pix] for the AOV.  rgbn == nullptr: every tile is one
// work item and writes its pixels itself.
struct PtSums {
    unsigned long long* rgbn;
    unsigned long long* depth;
};

struct TileShared {
    long long rgb[kBlock][3];
    long long depth[kBlock];
    unsigned int hits[kBlock], escapes[kBlock];
    unsigned int next;
};

__device__ __forceinline__ long long to_fixed(float v) { return __float2ll_rn(v * 4294967296.0f); }

// Delta-tracking path tracer (Section 4) over samples [s0, s1) of one tile of
// 256 pixels.  The work item's 256 (s1 - s0) paths (unit u = sample u / 256
// of tile pixel u % 256) are shared by the workgroup: every lane starts on one
// unit and takes the next one from an LDS counter when its path ends, so lanes
// on empty pixels or on short paths keep working.  Within a path the loop is flat: every iteration
// moves the lane to its next tentative collision and handles whatever event
// it reached (collision, escape, end of a shadow ray, start of a new path).
// The arithmetic and the random draws of each path are those of a recursive
// implementation: key (seed_lo ^ pixel, seed_hi), counter (block, sample,
// stream << 16 | bounce, frame).  Stream 0 of bounce b is path segment b:
// two draws for its direction (pixel jitter for b = 0, isotropic scattering
// otherwise), then its free flights and accept tests; stream 1 of bounce b is
// the shadow ray from collision b.  Results depend only on the pixel, not on
// the lane, tile shape or launch.
template <class Acc, bool AOV, bool ENV>
__device__ __forceinline__ void pt_tile(Acc& acc, int nx, int ny, int nz, const CameraK& cam,
                                        const MediumK& m, const PtArgs& g,
                                        const float* __restrict__ maj, const uint32_t* cbits,
                                        int bx, int by, TileShared& ts, const float4* tf_lds,
                                        float* __restrict__ image,
                                        float* __restrict__ aov, uint32_t& nsamp, uint32_t& ncell,
                                        uint32_t& nseg, uint32_t s0, uint32_t s1, PtSums sums)
{
    const int tid = threadIdx.x;
    const int tw = g.tw, th = 64 / g.tw;
    // the four waves sit side by side in one band of th rows: wave w covers
    // columns [x0 + w tw, x0 + (w + 1) tw), so the tile is 4 tw x th pixels
    // (256 x 1 at tw = 64: neighbouring waves trace neighbouring rays)
    const int x0 = bx * 4 * tw, y0 = by * th;
    ts.rgb[tid][0] = ts.rgb[tid][1] = ts.rgb[tid][2] = 0;
    ts.depth[tid] = 0;
    ts.hits[tid] = ts.escapes[tid] = 0;
    if (tid == 0) ts.next = (s0 + 1) * kBlock;
    __syncthreads();
    const uint32_t total = kBlock * s1;
    const float inv4pi = 0.0795774715459476679f;
    uint32_t u = s0 * kBlock + (uint32_t)tid;
    int q = 0, px = 0, py = 0;
    uint32_t k0 = 0, smp = 0;
    float L0 = 0.0f, L1 = 0.0f, L2 = 0.0f, b0 = 1.0f, b1 = 1.0f, b2 = 1.0f;
    float t0p = 0.0f, pdepth = 1.0f;
    bool phit = false;
    int b = 0;
    bool shadow = false, fresh = true;
    Rng rng;
    Flight f;
    while (u < total) {
        if (fresh) {
            q = (int)(u & (kBlock - 1));
            smp = u >> 8;
            const int w = q >> 6, l = q & 63;
            px = x0 + w * tw + (l % tw);
            py = y0 + (l / tw);
            if (px >= cam.width || py >= cam.height) {   // no pixel here
                u = atomicAdd(&ts.next, 1u);
                continue;
            }
            fresh = false;
            k0 = g.seed_lo ^ ((uint32_t)py * (uint32_t)cam.width + (uint32_t)px);
            rng.init(k0, g.seed_hi, smp, 0u, 0u, g.frame);
            const float jx = rng.next(), jy = rng.next();
            float o[3], d[3];
            camera_ray(cam, (float)px + jx, (float)py + jy, o, d);
            b = 0;
            shadow = false;
            L0 = L1 = L2 = 0.0f;
            b0 = b1 = b2 = 1.0f;
            flight_begin(f, g, nx, ny, nz, o, d, t0p);
            ++nseg;   // camera ray
        }
        const int tentative = flight_advance(f, maj, cbits, g, rng, ncell);
        if (tentative == kFlightYield) continue;
        // the density at the tentative collision is taken here, after the walk
        // loop, so that the lanes of a wave that reached one in different
        // steps of the walk sample in one pass
        float sv = 0.0f;
        if (tentative) {
            sv = trilinear(acc, fmaf(f.t, f.d[0], f.o[0]), fmaf(f.t, f.d[1], f.o[1]), fmaf(f.t, f.d[2], f.o[2]));
            ++nsamp;
        }
        const bool hit = tentative && rng.next() * f.mu < m.ds * tf_alpha_at(tf_lds, m, sv);
        if (tentative && !hit) continue;    // null collision: keep tracking
        bool path_done = false, next_bounce = false;
        if (!shadow) {
            if (b == 0) {
                phit = hit;
                pdepth = hit ? (f.t - t0p) / (f.t1 - t0p) : 1.0f;
            }
            if (hit) {
                // real collision: weight by albedo and colour, then the
                // shadow ray towards the light from the collision point
                const float4 c = tf_eval(m, sv);
                b0 *= m.albedo * c.x;
                b1 *= m.albedo * c.y;
                b2 *= m.albedo * c.z;
                const float x[3] = {fmaf(f.t, f.d[0], f.o[0]), fmaf(f.t, f.d[1], f.o[1]),
                                    fmaf(f.t, f.d[2], f.o[2])};
                rng.init(k0, g.seed_hi, smp, (uint32_t)b, 1u, g.frame);
                float t0s;
                flight_begin(f, g, nx, ny, nz, x, m.light, t0s);
                ++nseg;   // shadow ray
                shadow = true;
            } else {
                float e0, e1, e2;
                if (ENV) {   // the map's lookup only where a map is bound
                    escape_radiance(m, f.d, e0, e1, e2);
                } else {
                    e0 = m.ambient[0];
                    e1 = m.ambient[1];
                    e2 = m.ambient[2];
                }
                L0 = fmaf(b0, e0, L0);
                L1 = fmaf(b1, e1, L1);
                L2 = fmaf(b2, e2, L2);
                path_done = true;
            }
        } else {
            if (!hit) {
                L0 = fmaf(b0 * inv4pi, m.light_E[0], L0);
                L1 = fmaf(b1 * inv4pi, m.light_E[1], L1);
                L2 = fmaf(b2 * inv4pi, m.light_E[2], L2);
            }
            shadow = false;
            if (b + 1 == g.max_bounces) path_done = true;
            else next_bounce = true;
        }
        if (next_bounce) {
            // segment b + 1: isotropic scattering from the collision point
            // (the shadow ray's origin) with the first two draws of its
            // stream; with Russian roulette one survival draw comes first
            // (from bounce 2 on: survive with q = min(1, max throughput),
            // survivors carry throughput / q)
            ++b;
            rng.init(k0, g.seed_hi, smp, (uint32_t)b, 0u, g.frame);
            if (g.rr) {
                const float ur = rng.next();
                const float qs = b >= 2 ? fminf(fmaxf(fmaxf(b0, b1), b2), 1.0f) : 1.0f;
                if (ur < qs) {
                    b0 /= qs;
                    b1 /= qs;
                    b2 /= qs;
                } else {
                    path_done = true;
                }
            }
        }
        if (next_bounce && !path_done) {
            const float u1 = rng.next(), u2 = rng.next();
            const float z = 1.0f - 2.0f * u1;
            const float r = sqrtf(fmaxf(0.0f, 1.0f - z * z));
            const float phi = 6.28318530717958647692f * u2;
            const float o[3] = {f.o[0], f.o[1], f.o[2]};
            const float d[3] = {r * __cosf(phi), r * __sinf(phi), z};
            float t0n;
            flight_begin(f, g, nx, ny, nz, o, d, t0n);
            ++nseg;   // scattered ray
        }
        if (path_done) {
            atomicAdd(reinterpret_cast<unsigned long long*>(&ts.rgb[q][0]), (unsigned long long)to_fixed(L0));
            atomicAdd(reinterpret_cast<unsigned long long*>(&ts.rgb[q][1]), (unsigned long long)to_fixed(L1));
            atomicAdd(reinterpret_cast<unsigned long long*>(&ts.rgb[q][2]), (unsigned long long)to_fixed(L2));
            if (AOV) atomicAdd(reinterpret_cast<unsigned long long*>(&ts.depth[q]),
                               (unsigned long long)to_fixed(pdepth));
            atomicAdd(phit ? &ts.hits[q] : &ts.escapes[q], 1u);
            u = atomicAdd(&ts.next, 1u);
            fresh = true;
        }
    }
    __syncthreads();
    {
        const int w = tid >> 6, l = tid & 63;
        const int qx = x0 + w * tw + (l % tw), qy = y0 + (l / tw);
        if (qx < cam.width && qy < cam.height) {
            const uint32_t pix = (uint32_t)qy * (uint32_t)cam.width + (uint32_t)qx;
            if (sums.rgbn) {
                // integer sums: the total does not depend on the order in
                // which the tile's work items finish
                unsigned long long* a = sums.rgbn + 4 * (size_t)pix;
                atomicAdd(a + 0, (unsigned long long)ts.rgb[tid][0]);
                atomicAdd(a + 1, (unsigned long long)ts.rgb[tid][1]);
                atomicAdd(a + 2, (unsigned long long)ts.rgb[tid][2]);
                atomicAdd(a + 3, (unsigned long long)ts.hits[tid] | ((unsigned long long)ts.escapes[tid] << 32));
                if (AOV) atomicAdd(sums.depth + pix, (unsigned long long)ts.depth[tid]);
            } else {
                const double sc = 1.0 / (4294967296.0 * (double)g.spp);
                const float inv = 1.0f / (float)g.spp;
                reinterpret_cast<float4*>(image)[pix] =
                    make_float4((float)((double)ts.rgb[tid][0] * sc), (float)((double)ts.rgb[tid][1] * sc),
                                (float)((double)ts.rgb[tid][2] * sc), (float)ts.hits[tid] * inv);
                if (AOV)
                    reinterpret_cast<float2*>(aov)[pix] =
                        make_float2((float)((double)ts.depth[tid] * sc), (float)ts.escapes[tid] * inv);
            }
        }
    }
    __syncthreads();
}

// Clears the per-pixel sums of a split launch: n 16-byte words.
__global__ void pt_sums_clear_kernel(uint4* __restrict__ p, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// The image (and AOV) of a split launch from its per-pixel sums, with the
// scaling of the tiles that write their pixels themselves.
__global__ void pt_resolve_kernel(PtSums sums, float* __restrict__ image, float* __restrict__ aov, uint32_t npix,
                                  int spp)
{
    const uint32_t pix = blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= npix) return;
    const unsigned long long* a = sums.rgbn + 4 * (size_t)pix;
    const ulonglong2 rg = *reinterpret_cast<const ulonglong2*>(a);
    const ulonglong2 bn = *reinterpret_cast<const ulonglong2*>(a + 2);
    const double sc = 1.0 / (4294967296.0 * (double)spp);
    const float inv = 1.0f / (float)spp;
    reinterpret_cast<float4*>(image)[pix] =
        make_float4((float)((double)(long long)rg.x * sc), (float)((double)(long long)rg.y * sc),
                    (float)((double)(long long)bn.x * sc), (float)(unsigned int)(bn.y & 0xFFFFFFFFull) * inv);
    if (aov)
        reinterpret_cast<float2*>(aov)[pix] =
            make_float2((float)((double)(long long)sums.depth[pix] * sc), (float)(unsigned int)(bn.y >> 32) * inv);
}

// ---------------------------------------------------------------- cost order
// Optional order of the tiles in the work queue: most expensive first, so
// that the longest work items do not start last.  The estimate of a tile is
// the majorant optical depth of four camera rays through it (one through the
// middle of each wave tile, 32 midpoint steps across the volume's box),
// binned on a log scale (four bins per octave of 1 + depth, 64 bins); a
// counting sort over the bins gives the order.  Ties within a bin are taken
// in whatever order the atomics give: the image does not depend on the order.
constexpr int kCostBins = 64;

__global__ void pt_tile_cost_kernel(CameraK cam, PtArgs g, int nx, int ny, int nz, const float* __restrict__ maj,
                                    uint32_t tiles_x, uint32_t tiles, uint32_t* __restrict__ key,
                                    uint32_t* __restrict__ hist)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= tiles) return;
    const int tw = g.tw, th = 64 / g.tw;
    const float x0 = (float)((t % tiles_x) * 4u * (uint32_t)tw), y0 = (float)((t / tiles_x) * (uint32_t)th);
    float tau = 0.0f;
    for (int w = 0; w < 4; ++w) {
        float o[3], d[3], id[3], t0, t1;
        camera_ray(cam, x0 + ((float)w + 0.5f) * (float)tw, y0 + 0.5f * (float)th, o, d);
#pragma unroll
        for (int a = 0; a < 3; ++a) id[a] = 1.0f / d[a];
        if (!box_clip(nx, ny, nz, o, d, id, t0, t1)) continue;
        const float dt = (t1 - t0) * (1.0f / 32.0f);
        for (int k = 0; k < 32; ++k) {
            const float s = fmaf((float)k + 0.5f, dt, t0);
            const int cx = min(max((int)floorf((fmaf(s, d[0], o[0]) + 0.5f) * g.invC), 0), g.gx - 1);
            const int cy = min(max((int)floorf((fmaf(s, d[1], o[1]) + 0.5f) * g.invC), 0), g.gy - 1);
            const int cz = min(max((int)floorf((fmaf(s, d[2], o[2]) + 0.5f) * g.invC), 0), g.gz - 1);
            tau = fmaf(maj[cx + g.gx * (cy + g.gy * cz)], dt, tau);
        }
    }
    // fminf / fmaxf also map an infinite or NaN depth into the bin range
    const int k = (int)fmaxf(fminf(log2f(1.0f + fmaxf(tau, 0.0f)) * 4.0f, (float)(kCostBins - 1)), 0.0f);
    key[t] = (uint32_t)k;
    atomicAdd(&hist[k], 1u);
}

// First position of each bin in the queue, from the most expensive bin down.
__global__ void pt_cost_offsets_kernel(const uint32_t* __restrict__ hist, uint32_t* __restrict__ off)
{
    if (threadIdx.x != 0) return;
    uint32_t s = 0;
    for (int k = kCostBins - 1; k >= 0; --k) {
        off[k] = s;
        s += hist[k];
    }
}

__global__ void pt_cost_scatter_kernel(const uint32_t* __restrict__ key, uint32_t* __restrict__ off,
                                       uint32_t* __restrict__ order, uint32_t tiles)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= tiles) return;
    order[atomicAdd(&off[key[t]], 1u)] = t;
}

template <class Acc, class View, bool COUNT, bool AOV, bool ENV>
__global__ __launch_bounds__(kBlock, 4) void pt_kernel(View view, CameraK cam, MediumK m, PtArgs g,
                                                    const float* __restrict__ maj,
                                                    const uint32_t* __restrict__ coarse,
                                                    float* __restrict__ image,
                                                    float* __restrict__ aov,
                                                    unsigned long long* counter,
                                                    uint32_t* queue, PtSums sums,
                                                    const uint32_t* __restrict__ order)
{
    extern __shared__ uint32_t cbits[];
    __shared__ TileShared ts;
    for (int i = threadIdx.x; i < g.cwords; i += kBlock) cbits[i] = coarse[i];
    // the TF control points in LDS: every tentative collision reads two of them
    __shared__ float4 tf_lds[64];
    for (int i = threadIdx.x; i < m.tf_n; i += kBlock) tf_lds[i] = m.tf[i];
    __syncthreads();
    Acc acc{view};
    acc.reset();
    uint32_t nsamp = 0, ncell = 0, nseg = 0;
    // persistent workgroups take work items (tile, chunk of g.chunk samples)
    // from a queue, the tiles in raster order or in the given order, so a
    // workgroup that drew cheap items goes on to the next one at once, and
    // the paths of one expensive tile are spread over g.chunks workgroups
    __shared__ uint32_t s_item;
    const uint32_t tiles_x = (uint32_t)((cam.width + 4 * g.tw - 1) / (4 * g.tw));
    const uint32_t tiles = tiles_x * (uint32_t)((cam.height + 64 / g.tw - 1) / (64 / g.tw));
    const uint32_t items = tiles * g.chunks;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t it = s_item;   // pt_tile's barriers order this read before the next write
        if (it >= items) break;
        const uint32_t rank = it / g.chunks, s0 = (it % g.chunks) * g.chunk;
        const uint32_t t = order ? order[rank] : rank;
        pt_tile<Acc, AOV, ENV>(acc, view.nx, view.ny, view.nz, cam, m, g, maj, cbits, (int)(t % tiles_x),
                               (int)(t / tiles_x), ts, tf_lds, image, aov, nsamp, ncell, nseg, s0,
                               min(s0 + g.chunk, (uint32_t)g.spp), sums);
    }
    if (COUNT) {
        block_count(nsamp, counter);
        block_count(ncell, counter + 1);
        block_count(nseg, counter + 3);
    }
}

// ---------------------------------------------------------------- batched PT
// Many volumes in one persistent launch: workgroups pull (volume, work item)
// entries from an atomic counter over a list ordered by estimated cost
// (largest first) and render each item with the per-pixel code of pt_kernel,
// so every image is bit-identical to its own launch.  A volume's items are
// its tiles, or with g.chunks > 1 each tile's chunks of g.chunk samples
// (item = tile * g.chunks + chunk), which add into the volume's pixel sums.
struct BatchDesc {
    VdbView view;
    CameraK cam;
    MediumK med;
    PtArgs g;
    const float* maj;
    const uint32_t* coarse;
    float* image;
    PtSums sums;   // per-pixel integer sums when g.chunks > 1, else null
    int tiles_x;
};

__global__ void zero_u32(uint32_t* p)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0u;
}

__global__ __launch_bounds__(kBlock, 4) void pt_batch_kernel(const BatchDesc* __restrict__ descs,
                                                          const uint32_t* __restrict__ items,
                                                          uint32_t n_items, uint32_t* counter)
{
    extern __shared__ uint32_t cbits[];
    __shared__ uint32_t s_item;
    __shared__ TileShared ts;
    __shared__ float4 tf_lds[64];
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t it = __builtin_amdgcn_readfirstlane(s_item);
        if (it >= n_items) break;
        const uint32_t code = __builtin_amdgcn_readfirstlane(items[it]);
        const BatchDesc* D = descs + (code >> 20);
        const PtArgs g = D->g;
        const uint32_t sub = code & 0xFFFFFu;
        const uint32_t tile = sub / g.chunks, s0 = (sub % g.chunks) * g.chunk;
        const CameraK cam = D->cam;
        for (int i = threadIdx.x; i < g.cwords; i += kBlock) cbits[i] = D->coarse[i];
        for (int i = threadIdx.x; i < D->med.tf_n; i += kBlock) tf_lds[i] = D->med.tf[i];
        __syncthreads();
        VdbAcc acc{D->view};
        acc.reset();
        uint32_t ns = 0, nc = 0, nsg = 0;
        pt_tile<VdbAcc, false, true>(acc, D->view.nx, D->view.ny, D->view.nz, cam, D->med, g, D->maj, cbits,
                               (int)(tile % (uint32_t)D->tiles_x), (int)(tile / (uint32_t)D->tiles_x), ts,
                               tf_lds, D->image, nullptr, ns, nc, nsg, s0, min(s0 + g.chunk, (uint32_t)g.spp),
                               D->sums);
    }
}

}  // namespace vdbc
