// HIP kernels for gfx950 and their C-ABI launchers: sampling (Section 3.2.2),
// majorant macrocells, emission-absorption marching and the delta-tracking
// path tracer (Section 4), each for the compressed VDB and for the dense
// float32 baseline through the same templated code.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "common.h"
#include "device.h"
#include "format.h"
#include "host_header.h"

namespace vdbc {

constexpr int kTile = 16;          // 16x16 pixels per 256-thread workgroup
constexpr int kBlock = 256;
constexpr float kHddaEps = 1.0f / 64.0f;
// Upper bound on density evaluations in one free-flight search; a flight that
// reaches it is treated as escaping.  Only a majorant that exceeds the
// sampled extinction by many orders of magnitude can get near it.
constexpr uint32_t kMaxFlightSamples = 1u << 20;
// Macrocells a flight may enter in one iteration of the path loop before it
// yields (the walk resumes at the next iteration).  Lanes of a wave that walk
// long stretches of thin medium then wait at most this many DDA steps for the
// lanes that sample, instead of the whole walk.
constexpr int kWalkCells = 2;
// Value of flight_advance() when the flight yielded mid-walk.
constexpr int kFlightYield = 2;
// Resident PT workgroups per compute unit (the kernel's launch bounds).
constexpr int kPtBlocksPerCu = 4;

// ---------------------------------------------------------------- helpers

// 256 threads = 4 waves in a 2x2 arrangement, each wave a tw x (64/tw) pixel
// tile (tw = 8, 16, 32 or 64); workgroup (bx, by) covers a (2 tw) x (128/tw)
// block.  Returns false outside the image.
__device__ __forceinline__ bool tile_pixel(int width, int height, int tw, int bx, int by, int& px,
                                           int& py)
{
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, th = 64 / tw;
    px = bx * 2 * tw + (w & 1) * tw + (lane % tw);
    py = by * 2 * th + (w >> 1) * th + (lane / tw);
    return px < width && py < height;
}

// Adds a per-thread count to a global 64-bit counter, one atomic per block.
__device__ __forceinline__ void block_count(uint32_t n, unsigned long long* counter)
{
    __shared__ unsigned int s;
    if (threadIdx.x == 0) s = 0;
    __syncthreads();
    if (n) atomicAdd(&s, n);
    __syncthreads();
    if (threadIdx.x == 0 && s) atomicAdd(counter, (unsigned long long)s);
}

// Clears the workspace's counters: sample and cell counts, PT tile queue.
__global__ void zero_u64(unsigned long long* p)
{
    if (threadIdx.x < 3 && blockIdx.x == 0) p[threadIdx.x] = 0ull;
}

// ---------------------------------------------------------------- sampling

template <class Acc, class View>
__global__ __launch_bounds__(kBlock) void sample_kernel(View view, const float* __restrict__ pos,
                                                        uint64_t n, int filter,
                                                        float* __restrict__ out)
{
    Acc acc{view};
    acc.reset();
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    out[i] = filter ? trilinear(acc, x, y, z) : nearest(acc, x, y, z);
}

__global__ __launch_bounds__(kBlock) void lookup_kernel(VdbView view, const int32_t* __restrict__ ijk,
                                                        uint64_t n, float* __restrict__ out)
{
    VdbAcc acc{view};
    acc.reset();
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int x = ijk[3 * i], y = ijk[3 * i + 1], z = ijk[3 * i + 2];
    // voxels beyond the volume read B (edge leaves store B there, regions
    // past the last leaf or outside the root table resolve to B)
    out[i] = acc.voxel(x, y, z);
}

// ---------------------------------------------------------------- quality

// Error statistics of the compressed grid against the dense volume it was
// encoded from (the MSE / PSNR evaluation of Section 5.2).  A workgroup of
// 512 threads takes a 64 x 8 x 8 voxel region (eight leaves along x) in a
// grid-stride loop: thread (x, y) walks the region's 8 slices, so each wave
// reads 256 contiguous bytes of a dense row per slice and every thread stays
// in one leaf (one descent, then its leaf cache).  Per workgroup: {sum of
// squared differences, max |diff|, differing voxels, min dense, max dense}
// into part[5 * block]; a second kernel folds the partials in a fixed order
// (deterministic for a given size).
constexpr int kCmpThreads = 512;
constexpr int kCmpBlocks = 4096;

__global__ __launch_bounds__(kCmpThreads) void compare_kernel(VdbView view, const float* __restrict__ dense,
                                                              double* __restrict__ part)
{
    VdbAcc acc{view};
    acc.reset();
    const int t = threadIdx.x;
    const int lx = t & 63, ly = t >> 6;
    const uint64_t rx = (uint64_t)(view.nx + 63) / 64, ry = (uint64_t)(view.ny + 7) / 8,
                   rz = (uint64_t)(view.nz + 7) / 8;
    double sse = 0.0, mx = 0.0, nd = 0.0, lo = INFINITY, hi = -INFINITY;
    for (uint64_t r = blockIdx.x; r < rx * ry * rz; r += gridDim.x) {
        const int x = (int)(r % rx) * 64 + lx, y = (int)((r / rx) % ry) * 8 + ly;
        const int z0 = (int)(r / (rx * ry)) * 8;
        if (x >= view.nx || y >= view.ny) continue;
        for (int z = z0; z < z0 + 8 && z < view.nz; ++z) {
            const float dv =
                dense[(uint64_t)x + (uint64_t)view.nx * ((uint64_t)y + (uint64_t)view.ny * (uint64_t)z)];
            const float vv = acc.voxel(x, y, z);
            const double e = (double)vv - (double)dv;
            sse = fma(e, e, sse);
            mx = fmax(mx, fabs(e));
            nd += (__float_as_uint(vv) != __float_as_uint(dv)) ? 1.0 : 0.0;
            lo = fmin(lo, (double)dv);
            hi = fmax(hi, (double)dv);
        }
    }
    __shared__ double red[5][kCmpThreads];
    red[0][t] = sse;
    red[1][t] = mx;
    red[2][t] = nd;
    red[3][t] = lo;
    red[4][t] = hi;
    __syncthreads();
    for (int h = kCmpThreads / 2; h > 0; h >>= 1) {
        if (t < h) {
            red[0][t] += red[0][t + h];
            red[1][t] = fmax(red[1][t], red[1][t + h]);
            red[2][t] += red[2][t + h];
            red[3][t] = fmin(red[3][t], red[3][t + h]);
            red[4][t] = fmax(red[4][t], red[4][t + h]);
        }
        __syncthreads();
    }
    if (t < 5) part[5 * blockIdx.x + t] = red[t][0];
}

// Folds the per-workgroup partials: workgroup s reduces statistic s, each
// thread a fixed stride of partials, then a fixed-order tree in LDS.
__global__ __launch_bounds__(256) void compare_fold_kernel(const double* __restrict__ part, int blocks,
                                                           double* __restrict__ out)
{
    const int s = blockIdx.x, t = threadIdx.x;
    const bool sum = (s == 0 || s == 2), mn = (s == 3);
    double a = sum ? 0.0 : mn ? INFINITY : (s == 1 ? 0.0 : -INFINITY);
    for (int b = t; b < blocks; b += 256) {
        const double v = part[5 * b + s];
        a = sum ? a + v : mn ? fmin(a, v) : fmax(a, v);
    }
    __shared__ double red[256];
    red[t] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            const double v = red[t + h];
            red[t] = sum ? red[t] + v : mn ? fmin(red[t], v) : fmax(red[t], v);
        }
        __syncthreads();
    }
    if (t == 0) out[s] = red[0];
}

// ---------------------------------------------------------------- majorant

// One workgroup per macrocell: the 256 threads split the (C+2)^3 dilated
// footprint into z-columns (thread -> (i, j), walking k, so consecutive
// lookups stay in one leaf), then reduce min and max across the workgroup.
template <class Acc, class View>
__global__ __launch_bounds__(kBlock) void majorant_kernel(View view, MediumK m, int C, int gx,
                                                          int gy, int gz, float* __restrict__ out)
{
    Acc acc{view};
    acc.reset();
    const uint32_t cell = blockIdx.x;
    const int cx = (int)(cell % (uint32_t)gx), cy = (int)((cell / (uint32_t)gx) % (uint32_t)gy),
              cz = (int)(cell / ((uint32_t)gx * (uint32_t)gy));
    const int E = C + 2, x0 = C * cx - 1, y0 = C * cy - 1, z0 = C * cz - 1;
    float vmin = INFINITY, vmax = -INFINITY;
    for (int col = threadIdx.x; col < E * E; col += kBlock) {
        const int i = col % E, j = col / E;
        for (int k = 0; k < E; ++k) {
            const float v = acc.voxel(x0 + i, y0 + j, z0 + k);
            vmin = fminf(vmin, v);
            vmax = fmaxf(vmax, v);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        vmin = fminf(vmin, __shfl_xor(vmin, o));
        vmax = fmaxf(vmax, __shfl_xor(vmax, o));
    }
    __shared__ float red[2][kBlock / 64];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = vmin;
        red[1][w] = vmax;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int q = 1; q < kBlock / 64; ++q) {
        vmin = fminf(vmin, red[0][q]);
        vmax = fmaxf(vmax, red[1][q]);
    }
    // max of the piecewise-linear alpha over [vmin, vmax]: the two ends and
    // every control point strictly inside
    float a = fmaxf(tf_alpha(m, vmin), tf_alpha(m, vmax));
    const float p0 = (vmin - m.tf_lo) * m.tf_inv, p1 = (vmax - m.tf_lo) * m.tf_inv;
    for (int q = 0; q < m.tf_n; ++q)
        if ((float)q > p0 && (float)q < p1) a = fmaxf(a, m.tf[q].w);
    out[cell] = m.ds * a;
}

// ---------------------------------------------------------------- EA

template <class Acc, class View, bool HDDA, bool COUNT>
__global__ __launch_bounds__(kBlock) void ea_kernel(View view, CameraK cam, MediumK m, float step,
                                                    float t_term, float* __restrict__ image,
                                                    unsigned long long* counter)
{
    Acc acc{view};
    acc.reset();
    int px, py;
    const bool live = tile_pixel(cam.width, cam.height, 8, blockIdx.x, blockIdx.y, px, py);
    uint32_t nsamp = 0;
    if (live) {
        float o[3], d[3], t0, t1;
        camera_ray(cam, (float)px + 0.5f, (float)py + 0.5f, o, d);
        float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, T = 1.0f;
        const float id[3] = {1.0f / d[0], 1.0f / d[1], 1.0f / d[2]};
        if (box_clip(view.nx, view.ny, view.nz, o, d, id, t0, t1)) {
            for (int k = 0;; ++k) {
                const float t = fmaf((float)k + 0.5f, step, t0);
                if (t >= t1) break;
                const float x = fmaf(t, d[0], o[0]), y = fmaf(t, d[1], o[1]),
                            z = fmaf(t, d[2], o[2]);
                if (HDDA) {
                    const int i = (int)floorf(fmaxf(x, -2.0f)), j = (int)floorf(fmaxf(y, -2.0f)),
                              kk = (int)floorf(fmaxf(z, -2.0f));
                    const int L = acc.in_stored_leaf(i, j, kk) ? 0 : acc.empty_level(i, j, kk);
                    if (L) {
                        const int mask = (1 << L) - 1;
                        if ((i & mask) != mask && (j & mask) != mask && (kk & mask) != mask) {
                            // every sample whose footprint stays inside this
                            // empty node reads B with alpha 0: jump past it
                            const int lo[3] = {i & ~mask, j & ~mask, kk & ~mask};
                            float te = INFINITY;
#pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                if (d[a] > 0.0f)
                                    te = fminf(te, ((float)(lo[a] + mask) - kHddaEps - o[a]) / d[a]);
                                else if (d[a] < 0.0f)
                                    te = fminf(te, ((float)lo[a] + kHddaEps - o[a]) / d[a]);
                            }
                            const int kn = (int)floorf(fminf((te - t0) / step - 0.5f, 2.0e9f));
                            k = (kn > k + 1 ? kn : k + 1) - 1;
                            continue;
                        }
                    }
                }
                const float s = trilinear(acc, x, y, z);
                if (COUNT) ++nsamp;
                const float4 c = tf_eval(m, s);
                const float a = 1.0f - expf(-(m.ds * c.w) * step);
                const float ta = T * a;
                c0 = fmaf(ta, c.x, c0);
                c1 = fmaf(ta, c.y, c1);
                c2 = fmaf(ta, c.z, c2);
                T *= 1.0f - a;
                if (T < t_term) break;
            }
        }
        float4* img = reinterpret_cast<float4*>(image);
        img[(uint64_t)py * cam.width + px] = make_float4(c0, c1, c2, 1.0f - T);
    }
    if (COUNT) block_count(nsamp, counter);
}

// ---------------------------------------------------------------- ISO

// Implicit iso-surface marcher (the interval-based marcher of Section 5.4):
// the EA lattice t0 + (k + 1/2) step, the first pair of consecutive samples
// on opposite sides of the iso value (side: f >= iso), `refine` bisection
// steps on that interval, normal -grad f / |grad f| by central differences
// of half a voxel.  With HDDA, lattice samples whose trilinear footprint lies
// inside an empty node read B at every corner, so they take B's side without
// a field read; the crossing, the bisection and the image are unchanged.
template <class Acc, class View, bool HDDA, bool COUNT>
__global__ __launch_bounds__(kBlock) void iso_kernel(View view, CameraK cam, float iso, float step,
                                                     int refine, float* __restrict__ image,
                                                     float* __restrict__ aov,
                                                     unsigned long long* counter)
{
    Acc acc{view};
    acc.reset();
    int px, py;
    const bool live = tile_pixel(cam.width, cam.height, 8, blockIdx.x, blockIdx.y, px, py);
    uint32_t nsamp = 0;
    if (live) {
        float o[3], d[3], t0, t1;
        camera_ray(cam, (float)px + 0.5f, (float)py + 0.5f, o, d);
        float4 out = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        float thit = -1.0f;
        const float id[3] = {1.0f / d[0], 1.0f / d[1], 1.0f / d[2]};
        if (box_clip(view.nx, view.ny, view.nz, o, d, id, t0, t1)) {
            const bool bg_side = acc.background() >= iso;
            bool have = false, prev = false;
            float tprev = 0.0f;
            for (int k = 0;; ++k) {
                const float t = fmaf((float)k + 0.5f, step, t0);
                if (t >= t1) break;
                const float x = fmaf(t, d[0], o[0]), y = fmaf(t, d[1], o[1]), z = fmaf(t, d[2], o[2]);
                bool side;
                int last = k;   // last lattice sample of this step
                bool skip = false;
                if (HDDA) {
                    const int i = (int)floorf(fmaxf(x, -2.0f)), j = (int)floorf(fmaxf(y, -2.0f)),
                              kk = (int)floorf(fmaxf(z, -2.0f));
                    const int L = acc.in_stored_leaf(i, j, kk) ? 0 : acc.empty_level(i, j, kk);
                    if (L) {
                        const int mask = (1 << L) - 1;
                        if ((i & mask) != mask && (j & mask) != mask && (kk & mask) != mask) {
                            const int lo[3] = {i & ~mask, j & ~mask, kk & ~mask};
                            float te = INFINITY;
#pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                if (d[a] > 0.0f)
                                    te = fminf(te, ((float)(lo[a] + mask) - kHddaEps - o[a]) / d[a]);
                                else if (d[a] < 0.0f)
                                    te = fminf(te, ((float)lo[a] + kHddaEps - o[a]) / d[a]);
                            }
                            const int kn = (int)floorf(fminf((te - t0) / step - 0.5f, 2.0e9f));
                            last = (kn > k + 1 ? kn : k + 1) - 1;
                            skip = true;
                        }
                    }
                }
                if (skip) {
                    side = bg_side;
                } else {
                    side = trilinear(acc, x, y, z) >= iso;
                    if (COUNT) ++nsamp;
                }
                if (have && side != prev) {
                    // `refine` bisection steps, then the six central-difference
                    // samples of the normal, through one field evaluation
                    float lo = tprev, hi = t, mid = 0.0f;
                    float p0 = 0.0f, p1 = 0.0f, p2 = 0.0f, gx = 0.0f, gy = 0.0f, gz = 0.0f;
                    for (int it = 0; it < refine + 6; ++it) {
                        float q0, q1, q2;
                        const int e = it - refine;   // >= 0: gradient sample e
                        if (e < 0) {
                            mid = 0.5f * (lo + hi);
                            q0 = fmaf(mid, d[0], o[0]);
                            q1 = fmaf(mid, d[1], o[1]);
                            q2 = fmaf(mid, d[2], o[2]);
                        } else {
                            if (e == 0) {
                                thit = 0.5f * (lo + hi);
                                p0 = fmaf(thit, d[0], o[0]);
                                p1 = fmaf(thit, d[1], o[1]);
                                p2 = fmaf(thit, d[2], o[2]);
                            }
                            const float sh = (e & 1) ? -0.5f : 0.5f;
                            q0 = p0 + ((e >> 1) == 0 ? sh : 0.0f);
                            q1 = p1 + ((e >> 1) == 1 ? sh : 0.0f);
                            q2 = p2 + ((e >> 1) == 2 ? sh : 0.0f);
                        }
                        const float w = trilinear(acc, q0, q1, q2);
                        if (COUNT) ++nsamp;
                        if (e < 0) {
                            if ((w >= iso) == prev) lo = mid;
                            else hi = mid;
                        } else {
                            const float sw = (e & 1) ? -w : w;
                            if ((e >> 1) == 0) gx += sw;
                            else if ((e >> 1) == 1) gy += sw;
                            else gz += sw;
                        }
                    }
                    const float len = sqrtf(gx * gx + gy * gy + gz * gz);
                    out = len > 0.0f ? make_float4(0.5f * (1.0f - gx / len), 0.5f * (1.0f - gy / len),
                                                   0.5f * (1.0f - gz / len), 1.0f)
                                     : make_float4(0.5f, 0.5f, 0.5f, 1.0f);
                    break;
                }
                have = true;
                prev = side;
                tprev = last == k ? t : fmaf((float)last + 0.5f, step, t0);
                k = last;
            }
        }
        const uint64_t pix = (uint64_t)py * cam.width + px;
        reinterpret_cast<float4*>(image)[pix] = out;
        if (aov) reinterpret_cast<float2*>(aov)[pix] = make_float2(thit, 0.0f);
    }
    if (COUNT) block_count(nsamp, counter);
}

// ---------------------------------------------------------------- PT

struct PtArgs {
    int spp, max_bounces, C, gx, gy, gz, tw;
    float invC;
    int lf, cgx, cgy, cgz, cwords;   // coarse blocks of 2^lf macrocells per axis, bit words
    uint32_t seed_lo, seed_hi, frame;
    int rr;                          // Russian roulette from bounce 2 on
};

// Occupancy of the coarse blocks: bit set iff some macrocell of the block has
// a non-zero majorant.  One thread per block; a wave ballot assembles two
// 32-bit words per wave.
__global__ __launch_bounds__(kBlock) void coarse_bits_kernel(const float* __restrict__ maj,
                                                             PtArgs g, uint32_t* __restrict__ bits)
{
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
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
    const int w = (blockIdx.x * blockDim.x + threadIdx.x - lane) >> 5;   // first word of the wave
    if (lane == 0 && w < g.cwords) bits[w] = (uint32_t)ballot;
    if (lane == 0 && w + 1 < g.cwords) bits[w + 1] = (uint32_t)(ballot >> 32);
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
        f.id[a] = 1.0f / d[a];
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

// Advances the flight to its next tentative collision: returns 1 with the
// density `sv` sampled there (the caller makes the accept test), 0 when the
// segment leaves the grid without one, or kFlightYield after entering
// kWalkCells macrocells without a collision (call again to continue; the
// walk and its random draws are the same as without the pause).  Empty cells draw no random
// numbers and coarse-block faces are macrocell faces, so the tentative
// collisions are those of a uniform walk over every macrocell; a flight that
// overshoots a cell restarts at its exit (memorylessness).
template <class Acc>
__device__ __forceinline__ int flight_advance(Flight& f, Acc& acc, const MediumK& m,
                                              const float* __restrict__ maj,
                                              const uint32_t* cbits, const PtArgs& g, Rng& rng,
                                              float& sv, uint32_t& nsamp, uint32_t& ncell)
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
                sv = trilinear(acc, fmaf(f.t, f.d[0], f.o[0]), fmaf(f.t, f.d[1], f.o[1]),
                               fmaf(f.t, f.d[2], f.o[2]));
                ++nsamp;
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
            f.imu = 1.0f / f.mu;
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
struct TileShared {
    long long rgb[kBlock][3];
    long long depth[kBlock];
    unsigned int hits[kBlock], escapes[kBlock];
    unsigned int next;
};

__device__ __forceinline__ long long to_fixed(float v) { return __float2ll_rn(v * 4294967296.0f); }

// Delta-tracking path tracer (Section 4) over one tile of 256 pixels.  The
// tile's 256 x spp paths (unit u = sample u / 256 of tile pixel u % 256) are
// shared by the workgroup: every lane starts on one unit and takes the next
// one from an LDS counter when its path ends, so lanes on empty pixels or on
// short paths keep working.  Within a path the loop is flat: every iteration
// moves the lane to its next tentative collision and handles whatever event
// it reached (collision, escape, end of a shadow ray, start of a new path).
// The arithmetic and the random draws of each path are those of a recursive
// implementation: key (seed_lo ^ pixel, seed_hi), counter (block, sample,
// stream << 16 | bounce, frame).  Stream 0 of bounce b is path segment b:
// two draws for its direction (pixel jitter for b = 0, isotropic scattering
// otherwise), then its free flights and accept tests; stream 1 of bounce b is
// the shadow ray from collision b.  Results depend only on the pixel, not on
// the lane, tile shape or launch.
template <class Acc, bool AOV>
__device__ __forceinline__ void pt_tile(Acc& acc, int nx, int ny, int nz, const CameraK& cam,
                                        const MediumK& m, const PtArgs& g,
                                        const float* __restrict__ maj, const uint32_t* cbits,
                                        int bx, int by, TileShared& ts, float* __restrict__ image,
                                        float* __restrict__ aov, uint32_t& nsamp, uint32_t& ncell)
{
    const int tid = threadIdx.x;
    const int tw = g.tw, th = 64 / g.tw;
    const int x0 = bx * 2 * tw, y0 = by * 2 * th;
    ts.rgb[tid][0] = ts.rgb[tid][1] = ts.rgb[tid][2] = 0;
    ts.depth[tid] = 0;
    ts.hits[tid] = ts.escapes[tid] = 0;
    if (tid == 0) ts.next = kBlock;
    __syncthreads();
    const uint32_t total = (uint32_t)kBlock * (uint32_t)g.spp;
    const float inv4pi = 0.0795774715459476679f;
    uint32_t u = (uint32_t)tid;
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
            px = x0 + (w & 1) * tw + (l % tw);
            py = y0 + (w >> 1) * th + (l / tw);
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
        }
        float sv = 0.0f;
        const int tentative = flight_advance(f, acc, m, maj, cbits, g, rng, sv, nsamp, ncell);
        if (tentative == kFlightYield) continue;
        const bool hit = tentative && rng.next() * f.mu < m.ds * tf_alpha(m, sv);
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
                shadow = true;
            } else {
                L0 = fmaf(b0, m.ambient[0], L0);
                L1 = fmaf(b1, m.ambient[1], L1);
                L2 = fmaf(b2, m.ambient[2], L2);
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
        const int qx = x0 + (w & 1) * tw + (l % tw), qy = y0 + (w >> 1) * th + (l / tw);
        if (qx < cam.width && qy < cam.height) {
            const uint32_t pix = (uint32_t)qy * (uint32_t)cam.width + (uint32_t)qx;
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
    __syncthreads();
}

template <class Acc, class View, bool COUNT, bool AOV>
__global__ __launch_bounds__(kBlock, 4) void pt_kernel(View view, CameraK cam, MediumK m, PtArgs g,
                                                    const float* __restrict__ maj,
                                                    const uint32_t* __restrict__ coarse,
                                                    float* __restrict__ image,
                                                    float* __restrict__ aov,
                                                    unsigned long long* counter,
                                                    uint32_t* queue)
{
    extern __shared__ uint32_t cbits[];
    __shared__ TileShared ts;
    for (int i = threadIdx.x; i < g.cwords; i += kBlock) cbits[i] = coarse[i];
    __syncthreads();
    Acc acc{view};
    acc.reset();
    uint32_t nsamp = 0, ncell = 0;
    // persistent workgroups take tiles in raster order from a queue, so a
    // workgroup that drew cheap tiles goes on to the next one at once
    __shared__ uint32_t s_tile;
    const uint32_t tiles_x = (uint32_t)((cam.width + 2 * g.tw - 1) / (2 * g.tw));
    const uint32_t tiles = tiles_x * (uint32_t)((cam.height + 128 / g.tw - 1) / (128 / g.tw));
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t t = s_tile;   // pt_tile's barriers order this read before the next write
        if (t >= tiles) break;
        pt_tile<Acc, AOV>(acc, view.nx, view.ny, view.nz, cam, m, g, maj, cbits, (int)(t % tiles_x),
                          (int)(t / tiles_x), ts, image, aov, nsamp, ncell);
    }
    if (COUNT) {
        block_count(nsamp, counter);
        block_count(ncell, counter + 1);
    }
}

// ---------------------------------------------------------------- batched PT
// Many volumes in one persistent launch: workgroups pull (volume, tile) items
// from an atomic counter over a list ordered by estimated cost (largest
// first) and render each tile with the per-pixel code of pt_kernel, so every
// image is bit-identical to its own launch.
struct BatchDesc {
    VdbView view;
    CameraK cam;
    MediumK med;
    PtArgs g;
    const float* maj;
    const uint32_t* coarse;
    float* image;
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
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t it = __builtin_amdgcn_readfirstlane(s_item);
        if (it >= n_items) break;
        const uint32_t code = __builtin_amdgcn_readfirstlane(items[it]);
        const BatchDesc* D = descs + (code >> 20);
        const uint32_t tile = code & 0xFFFFFu;
        const PtArgs g = D->g;
        const CameraK cam = D->cam;
        for (int i = threadIdx.x; i < g.cwords; i += kBlock) cbits[i] = D->coarse[i];
        __syncthreads();
        VdbAcc acc{D->view};
        acc.reset();
        uint32_t ns = 0, nc = 0;
        pt_tile<VdbAcc, false>(acc, D->view.nx, D->view.ny, D->view.nz, cam, D->med, g, D->maj, cbits,
                               (int)(tile % (uint32_t)D->tiles_x), (int)(tile / (uint32_t)D->tiles_x), ts,
                               D->image, nullptr, ns, nc);
    }
}

__global__ void philox_kernel(const uint32_t* __restrict__ ctr, const uint32_t* __restrict__ key,
                              uint64_t n, uint32_t* __restrict__ out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c0 = ctr[4 * i], c1 = ctr[4 * i + 1], c2 = ctr[4 * i + 2], c3 = ctr[4 * i + 3];
    philox4x32_10(c0, c1, c2, c3, key[2 * i], key[2 * i + 1]);
    out[4 * i] = c0;
    out[4 * i + 1] = c1;
    out[4 * i + 2] = c2;
    out[4 * i + 3] = c3;
}

// ---------------------------------------------------------------- host side

static vdbc_status launch_check(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VDBC_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
    return VDBC_OK;
}

static vdbc_status make_view(const vdbc_grid* g, VdbView* v)
{
    if (!g || !g->device) return fail(VDBC_E_INVALID, "null grid");
    Header h;
    vdbc_status s = parse_header(g->header, g->bytes, &h);
    if (s) return s;
    const uint8_t* b = static_cast<const uint8_t*>(g->device);
    v->root = reinterpret_cast<const uint32_t*>(b + h.off_root);
    v->upper = reinterpret_cast<const Word*>(b + h.off_upper);
    v->lower = reinterpret_cast<const Word*>(b + h.off_lower);
    v->upper_tiles = reinterpret_cast<const float*>(b + h.off_upper_tiles);
    v->lower_tiles = reinterpret_cast<const float*>(b + h.off_lower_tiles);
    v->leaf_values = reinterpret_cast<const float*>(b + h.off_leaf_values);
    v->bg = reinterpret_cast<const float*>(b + hdr::background);
    v->nx = (int)h.nx;
    v->ny = (int)h.ny;
    v->nz = (int)h.nz;
    v->rnx = (int)h.root_nx;
    v->rny = (int)h.root_ny;
    v->rnz = (int)h.root_nz;
    v->background = h.background;
    return VDBC_OK;
}

static vdbc_status make_dense(const float* dense, vdbc_dims d, float background, DenseView* v)
{
    if (!dense) return fail(VDBC_E_INVALID, "null dense array");
    if (d.nx == 0 || d.ny == 0 || d.nz == 0 || d.nx > 0x7FFFFFFFu || d.ny > 0x7FFFFFFFu ||
        d.nz > 0x7FFFFFFFu)
        return fail(VDBC_E_INVALID, "dims must be in [1, 2^31)");
    if (!std::isfinite(background)) return fail(VDBC_E_INVALID, "background must be finite");
    v->data = dense;
    v->nx = (int)d.nx;
    v->ny = (int)d.ny;
    v->nz = (int)d.nz;
    v->background = background;
    return VDBC_OK;
}

static vdbc_status make_medium(const vdbc_medium* m, int nx, int ny, int nz, MediumK* k)
{
    if (!m) return fail(VDBC_E_INVALID, "null medium");
    if (m->tf_n < 2 || m->tf_n > 64) return fail(VDBC_E_INVALID, "tf_n must be in [2, 64]");
    if (!(m->tf_hi > m->tf_lo) || !std::isfinite(m->tf_lo) || !std::isfinite(m->tf_hi))
        return fail(VDBC_E_INVALID, "need finite tf_lo < tf_hi");
    if (!std::isfinite(m->sigma_scale) || m->sigma_scale < 0.0f)
        return fail(VDBC_E_INVALID, "sigma_scale must be finite and >= 0");
    std::memset(k, 0, sizeof *k);
    const int nmax = nx > ny ? (nx > nz ? nx : nz) : (ny > nz ? ny : nz);
    k->ds = m->sigma_scale / (float)nmax;
    k->albedo = m->albedo;
    k->tf_n = (int)m->tf_n;
    k->tf_lo = m->tf_lo;
    k->tf_inv = (float)(m->tf_n - 1) / (m->tf_hi - m->tf_lo);
    for (uint32_t i = 0; i < m->tf_n; ++i) {
        for (int c = 0; c < 4; ++c)
            if (!std::isfinite(m->tf[i][c])) return fail(VDBC_E_INVALID, "non-finite TF entry");
        if (m->tf[i][3] < 0.0f) return fail(VDBC_E_INVALID, "TF alpha must be >= 0");
        k->tf[i] = make_float4(m->tf[i][0], m->tf[i][1], m->tf[i][2], m->tf[i][3]);
    }
    for (int a = 0; a < 3; ++a) {
        k->light[a] = m->light_dir[a];
        k->light_E[a] = m->light_E[a];
        k->ambient[a] = m->ambient[a];
    }
    return VDBC_OK;
}

// Host mirror of the device TF alpha (for the HDDA precondition alpha(B)=0).
static float host_alpha(const MediumK& m, float s)
{
    float pos = (s - m.tf_lo) * m.tf_inv;
    pos = std::fmin(std::fmax(pos, 0.0f), (float)(m.tf_n - 1));
    int i = (int)pos;
    i = i > m.tf_n - 2 ? m.tf_n - 2 : i;
    const float fr = pos - (float)i;
    return std::fma(fr, m.tf[i + 1].w - m.tf[i].w, m.tf[i].w);
}

static vdbc_status make_camera(const vdbc_camera* c, CameraK* k)
{
    if (!c) return fail(VDBC_E_INVALID, "null camera");
    if (c->kind > 1) return fail(VDBC_E_INVALID, "camera kind must be 0 or 1");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(c->origin[a]) || !std::isfinite(c->lower_left[a]) ||
            !std::isfinite(c->du[a]) || !std::isfinite(c->dv[a]) || !std::isfinite(c->dir[a]))
            return fail(VDBC_E_INVALID, "non-finite camera vector");
    if (c->kind == 0 && c->dir[0] == 0.0f && c->dir[1] == 0.0f && c->dir[2] == 0.0f)
        return fail(VDBC_E_INVALID, "orthographic camera needs a non-zero direction");
    if (c->width == 0 || c->height == 0 || c->width > 65536 * kTile || c->height > 65535u * kTile)
        return fail(VDBC_E_INVALID, "bad image size");
    k->kind = (int)c->kind;
    k->width = (int)c->width;
    k->height = (int)c->height;
    for (int a = 0; a < 3; ++a) {
        k->o[a] = c->origin[a];
        k->ll[a] = c->lower_left[a];
        k->du[a] = c->du[a];
        k->dv[a] = c->dv[a];
        k->dir[a] = c->dir[a];
    }
    return VDBC_OK;
}

static uint64_t majorant_bytes(uint32_t C, int nx, int ny, int nz)
{
    const uint64_t gx = (nx + C - 1) / C, gy = (ny + C - 1) / C, gz = (nz + C - 1) / C;
    return gx * gy * gz * 4u;
}

// Majorant grid and coarse occupancy geometry.  Coarse blocks are 2^lf
// macrocells per axis, the largest power of two spanning at most 32 voxels (one
// brick), doubled until the bit mask fits in 32 KB of LDS.
static void pt_geometry(uint32_t C, int nx, int ny, int nz, PtArgs* g)
{
    g->C = (int)C;
    g->invC = 1.0f / (float)C;
    g->gx = (nx + g->C - 1) / g->C;
    g->gy = (ny + g->C - 1) / g->C;
    g->gz = (nz + g->C - 1) / g->C;
    int lf = 0;
    while ((C << (lf + 1)) <= 32) ++lf;      // block edge C * 2^lf <= 32 voxels
    for (;;) {
        const int F = 1 << lf;
        g->lf = lf;
        g->cgx = (g->gx + F - 1) / F;
        g->cgy = (g->gy + F - 1) / F;
        g->cgz = (g->gz + F - 1) / F;
        const uint64_t cells = (uint64_t)g->cgx * g->cgy * g->cgz;
        g->cwords = (int)((cells + 31) / 32);
        if (g->cwords <= 8192) break;
        ++lf;
    }
}

static uint64_t pt_workspace(uint32_t C, int nx, int ny, int nz)
{
    PtArgs g;
    pt_geometry(C, nx, ny, nz, &g);
    return 256 + align256(majorant_bytes(C, nx, ny, nz)) + align256(4ull * g.cwords);
}

static vdbc_status check_samples(const float* pos, uint64_t n, uint32_t filter, float* out)
{
    if (filter > 1) return fail(VDBC_E_INVALID, "filter must be 0 or 1");
    if (n && (!pos || !out)) return fail(VDBC_E_INVALID, "null positions or output");
    if (n > (uint64_t)0x7FFFFFFFull * kBlock) return fail(VDBC_E_INVALID, "too many samples");
    return VDBC_OK;
}

template <class Acc, class View>
static vdbc_status launch_majorant(const View& v, const MediumK& m, uint32_t C, float* out,
                                   hipStream_t st)
{
    const int gx = (v.nx + C - 1) / C, gy = (v.ny + C - 1) / C, gz = (v.nz + C - 1) / C;
    const uint64_t cells = (uint64_t)gx * gy * gz;
    if (cells > 0x7FFFFFFFull) return fail(VDBC_E_INVALID, "too many macrocells (%llu)", (unsigned long long)cells);
    hipLaunchKernelGGL((majorant_kernel<Acc, View>), dim3((unsigned)cells), dim3(kBlock), 0, st, v, m,
                       (int)C, gx, gy, gz, out);
    return launch_check("majorant");
}

// Compute units of the current device (cached per device; 256 if unknown).
static int device_cus()
{
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 256;
    if (dev < 64 && cache[dev].load(std::memory_order_relaxed) > 0)
        return cache[dev].load(std::memory_order_relaxed);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    if (dev < 64) cache[dev].store(cus, std::memory_order_relaxed);
    return cus;
}

template <class Acc, class View>
static vdbc_status render_impl(const View& v, const vdbc_camera* c, const vdbc_medium* med,
                               const vdbc_render_params* r, float* image, float* aov, void* ws,
                               uint64_t ws_bytes, void* stream)
{
    if (!r || !image) return fail(VDBC_E_INVALID, "null params or image");
    CameraK cam;
    MediumK m;
    vdbc_status s = make_camera(c, &cam);
    if (s) return s;
    if (r->mode > 2) return fail(VDBC_E_INVALID, "mode must be EA (0), PT (1) or ISO (2)");
    if (r->mode != VDBC_MODE_ISO) {
        s = make_medium(med, v.nx, v.ny, v.nz, &m);
        if (s) return s;
    }
    const bool count = (r->flags & VDBC_RENDER_COUNT) != 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned long long* counter = reinterpret_cast<unsigned long long*>(ws);
    vdbc_dims d{(uint32_t)v.nx, (uint32_t)v.ny, (uint32_t)v.nz};
    uint64_t need = 0;
    s = vdbc_render_workspace(r, d, &need);
    if (s) return s;
    if (need && (!ws || ws_bytes < need))
        return fail(VDBC_E_BUFFER_TOO_SMALL, "workspace needs %llu bytes", (unsigned long long)need);
    if (ws && reinterpret_cast<uintptr_t>(ws) % 256)
        return fail(VDBC_E_INVALID, "workspace must be 256-byte aligned");
    dim3 grid((cam.width + kTile - 1) / kTile, (cam.height + kTile - 1) / kTile);
    if (r->mode == VDBC_MODE_ISO) {
        if (!(r->step > 0.0f) || !std::isfinite(r->step))
            return fail(VDBC_E_INVALID, "ISO step must be finite and > 0");
        const double diag = std::sqrt((double)v.nx * v.nx + (double)v.ny * v.ny + (double)v.nz * v.nz);
        if (diag / r->step > 16777216.0)
            return fail(VDBC_E_INVALID, "ISO step too small for this volume (> 2^24 samples per ray)");
        if (!std::isfinite(r->iso)) return fail(VDBC_E_INVALID, "iso value must be finite");
        if (r->refine > 64) return fail(VDBC_E_INVALID, "refine must be <= 64");
        if (count) {
            hipLaunchKernelGGL(zero_u64, dim3(1), dim3(64), 0, st, counter);
            if ((s = launch_check("zero counter"))) return s;
        }
        const bool hdda = (r->flags & VDBC_RENDER_HDDA) != 0;
#define ISO_LAUNCH(H, CNT)                                                                      \
    hipLaunchKernelGGL((iso_kernel<Acc, View, H, CNT>), grid, dim3(kBlock), 0, st, v, cam, r->iso, \
                       r->step, (int)r->refine, image, aov, counter)
        if (hdda) {
            if (count) ISO_LAUNCH(true, true);
            else ISO_LAUNCH(true, false);
        } else {
            if (count) ISO_LAUNCH(false, true);
            else ISO_LAUNCH(false, false);
        }
#undef ISO_LAUNCH
        return launch_check("iso render");
    }
    if (count && r->mode == VDBC_MODE_EA) {
        hipLaunchKernelGGL(zero_u64, dim3(1), dim3(64), 0, st, counter);
        if ((s = launch_check("zero counter"))) return s;
    }
    if (r->mode == VDBC_MODE_EA) {
        if (!(r->step > 0.0f) || !std::isfinite(r->step))
            return fail(VDBC_E_INVALID, "EA step must be finite and > 0");
        // bound the per-ray loop: box diagonal / step <= 2^24 samples
        const double diag = std::sqrt((double)v.nx * v.nx + (double)v.ny * v.ny + (double)v.nz * v.nz);
        if (diag / r->step > 16777216.0)
            return fail(VDBC_E_INVALID, "EA step too small for this volume (> 2^24 samples per ray)");
        const bool hdda = (r->flags & VDBC_RENDER_HDDA) && host_alpha(m, v.background) == 0.0f;
#define EA_LAUNCH(H, CNT)                                                                      \
    hipLaunchKernelGGL((ea_kernel<Acc, View, H, CNT>), grid, dim3(kBlock), 0, st, v, cam, m, \
                       r->step, r->t_terminate, image, counter)
        if (hdda) {
            if (count) EA_LAUNCH(true, true);
            else EA_LAUNCH(true, false);
        } else {
            if (count) EA_LAUNCH(false, true);
            else EA_LAUNCH(false, false);
        }
#undef EA_LAUNCH
        return launch_check("ea render");
    }
    if (r->spp == 0 || r->max_bounces == 0) return fail(VDBC_E_INVALID, "spp and max_bounces must be >= 1");
    {
        const double l = std::sqrt((double)med->light_dir[0] * med->light_dir[0] +
                                   (double)med->light_dir[1] * med->light_dir[1] +
                                   (double)med->light_dir[2] * med->light_dir[2]);
        if (!(std::fabs(l - 1.0) <= 1e-3)) return fail(VDBC_E_INVALID, "light_dir must be a unit vector");
        if (!std::isfinite(med->albedo) || med->albedo < 0.0f)
            return fail(VDBC_E_INVALID, "albedo must be finite and >= 0");
    }
    hipLaunchKernelGGL(zero_u64, dim3(1), dim3(64), 0, st, counter);   // counters and tile queue
    if ((s = launch_check("zero counters"))) return s;
    float* maj = reinterpret_cast<float*>(static_cast<uint8_t*>(ws) + 256);
    if (!(r->flags & VDBC_RENDER_KEEP_MAJORANT)) {
        s = launch_majorant<Acc>(v, m, r->macrocell, maj, st);
        if (s) return s;
    }
    PtArgs g;
    pt_geometry(r->macrocell, v.nx, v.ny, v.nz, &g);
    g.spp = (int)r->spp;
    g.max_bounces = (int)r->max_bounces;
    g.tw = (r->tile_w == 16 || r->tile_w == 32 || r->tile_w == 64) ? (int)r->tile_w : 8;
    g.seed_lo = (uint32_t)r->seed;
    g.seed_hi = (uint32_t)(r->seed >> 32);
    g.frame = r->frame;
    g.rr = (r->flags & VDBC_RENDER_RR) ? 1 : 0;
    uint32_t* coarse = reinterpret_cast<uint32_t*>(
        static_cast<uint8_t*>(ws) + 256 + align256(majorant_bytes(r->macrocell, v.nx, v.ny, v.nz)));
    {
        const uint64_t ncoarse = (uint64_t)g.cgx * g.cgy * g.cgz;
        hipLaunchKernelGGL(coarse_bits_kernel, dim3((unsigned)((ncoarse + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, st, maj, g, coarse);
        if ((s = launch_check("coarse occupancy"))) return s;
    }
    const size_t lds = 4u * (size_t)g.cwords;
    {
        const uint64_t tiles = (uint64_t)((cam.width + 2 * g.tw - 1) / (2 * g.tw)) *
                               (uint64_t)((cam.height + 128 / g.tw - 1) / (128 / g.tw));
        grid = dim3((unsigned)std::min<uint64_t>(tiles, (uint64_t)device_cus() * kPtBlocksPerCu));
    }
    uint32_t* queue = reinterpret_cast<uint32_t*>(counter + 2);
#define PT_LAUNCH(CNT, AO)                                                                     \
    hipLaunchKernelGGL((pt_kernel<Acc, View, CNT, AO>), grid, dim3(kBlock), lds, st, v, cam, m, \
                       g, maj, coarse, image, aov, counter, queue)
    if (count) {
        if (aov) PT_LAUNCH(true, true);
        else PT_LAUNCH(true, false);
    } else {
        if (aov) PT_LAUNCH(false, true);
        else PT_LAUNCH(false, false);
    }
#undef PT_LAUNCH
    return launch_check("pt render");
}

}  // namespace vdbc

using namespace vdbc;

extern "C" vdbc_status vdbc_sample(const vdbc_grid* g, const float* pos, uint64_t n,
                                   uint32_t filter, float* out, void* stream)
{
    clear_error();
    VdbView v;
    vdbc_status s = make_view(g, &v);
    if (s) return s;
    if ((s = check_samples(pos, n, filter, out))) return s;
    if (n == 0) return VDBC_OK;
    hipLaunchKernelGGL((sample_kernel<VdbAcc, VdbView>), dim3((unsigned)((n + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, static_cast<hipStream_t>(stream), v, pos, n, (int)filter, out);
    return launch_check("vdbc_sample");
}

extern "C" vdbc_status vdbc_sample_dense(const float* dense, vdbc_dims d, float background,
                                         const float* pos, uint64_t n, uint32_t filter, float* out,
                                         void* stream)
{
    clear_error();
    DenseView v;
    vdbc_status s = make_dense(dense, d, background, &v);
    if (s) return s;
    if ((s = check_samples(pos, n, filter, out))) return s;
    if (n == 0) return VDBC_OK;
    hipLaunchKernelGGL((sample_kernel<DenseAcc, DenseView>),
                       dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       static_cast<hipStream_t>(stream), v, pos, n, (int)filter, out);
    return launch_check("vdbc_sample_dense");
}

extern "C" vdbc_status vdbc_lookup(const vdbc_grid* g, const int32_t* ijk, uint64_t n, float* out,
                                   void* stream)
{
    clear_error();
    VdbView v;
    vdbc_status s = make_view(g, &v);
    if (s) return s;
    if (n && (!ijk || !out)) return fail(VDBC_E_INVALID, "null coordinates or output");
    if (n > (uint64_t)0x7FFFFFFFull * kBlock) return fail(VDBC_E_INVALID, "too many lookups");
    if (n == 0) return VDBC_OK;
    hipLaunchKernelGGL(lookup_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       static_cast<hipStream_t>(stream), v, ijk, n, out);
    return launch_check("vdbc_lookup");
}

static uint64_t compare_regions(uint64_t nx, uint64_t ny, uint64_t nz)
{
    return ((nx + 63) / 64) * ((ny + 7) / 8) * ((nz + 7) / 8);
}

static uint32_t compare_blocks(const VdbView& v)
{
    const uint64_t regions = compare_regions((uint64_t)v.nx, (uint64_t)v.ny, (uint64_t)v.nz);
    return (uint32_t)std::min<uint64_t>(regions, kCmpBlocks);
}

extern "C" vdbc_status vdbc_compare_workspace(vdbc_dims d, uint64_t* bytes)
{
    clear_error();
    if (!bytes) return fail(VDBC_E_INVALID, "null argument");
    if (d.nx == 0 || d.ny == 0 || d.nz == 0) return fail(VDBC_E_INVALID, "zero dims");
    const uint64_t regions = compare_regions(d.nx, d.ny, d.nz);
    *bytes = 5ull * 8ull * std::min<uint64_t>(regions, kCmpBlocks);
    return VDBC_OK;
}

extern "C" vdbc_status vdbc_compare_dense(const vdbc_grid* g, const float* dense, double* out, void* ws,
                                          uint64_t ws_bytes, void* stream)
{
    clear_error();
    VdbView v;
    vdbc_status s = make_view(g, &v);
    if (s) return s;
    if (!dense || !out) return fail(VDBC_E_INVALID, "null dense volume or output");
    const uint32_t blocks = compare_blocks(v);
    if (!ws || ws_bytes < 40ull * blocks)
        return fail(VDBC_E_BUFFER_TOO_SMALL, "workspace needs %llu bytes", 40ull * blocks);
    if (reinterpret_cast<uintptr_t>(ws) % 8) return fail(VDBC_E_INVALID, "workspace must be 8-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    double* part = static_cast<double*>(ws);
    hipLaunchKernelGGL(compare_kernel, dim3(blocks), dim3(kCmpThreads), 0, st, v, dense, part);
    if ((s = launch_check("compare"))) return s;
    hipLaunchKernelGGL(compare_fold_kernel, dim3(5), dim3(256), 0, st, part, (int)blocks, out);
    return launch_check("compare fold");
}

extern "C" vdbc_status vdbc_render_workspace(const vdbc_render_params* r, vdbc_dims d,
                                             uint64_t* bytes)
{
    if (!r || !bytes) return fail(VDBC_E_INVALID, "null argument");
    if (d.nx == 0 || d.ny == 0 || d.nz == 0) return fail(VDBC_E_INVALID, "zero dims");
    if (r->mode == VDBC_MODE_PT) {
        if (r->macrocell < 4 || r->macrocell > 64 || (r->macrocell & (r->macrocell - 1)))
            return fail(VDBC_E_INVALID, "macrocell must be 4, 8, 16, 32 or 64");
        *bytes = pt_workspace(r->macrocell, (int)d.nx, (int)d.ny, (int)d.nz);
    } else {
        *bytes = (r->flags & VDBC_RENDER_COUNT) ? 256 : 0;
    }
    return VDBC_OK;
}

extern "C" vdbc_status vdbc_render(const vdbc_grid* g, const vdbc_camera* c, const vdbc_medium* m,
                                   const vdbc_render_params* r, float* image, float* aov, void* ws,
                                   uint64_t ws_bytes, void* stream)
{
    clear_error();
    VdbView v;
    vdbc_status s = make_view(g, &v);
    if (s) return s;
    return render_impl<VdbAcc>(v, c, m, r, image, aov, ws, ws_bytes, stream);
}

extern "C" vdbc_status vdbc_render_dense(const float* dense, vdbc_dims d, float background,
                                         const vdbc_camera* c, const vdbc_medium* m,
                                         const vdbc_render_params* r, float* image, float* aov,
                                         void* ws, uint64_t ws_bytes, void* stream)
{
    clear_error();
    DenseView v;
    vdbc_status s = make_dense(dense, d, background, &v);
    if (s) return s;
    return render_impl<DenseAcc>(v, c, m, r, image, aov, ws, ws_bytes, stream);
}

extern "C" vdbc_status vdbc_majorant(const vdbc_grid* g, const vdbc_medium* med, uint32_t C,
                                     float* out, void* stream)
{
    clear_error();
    VdbView v;
    vdbc_status s = make_view(g, &v);
    if (s) return s;
    if (!out) return fail(VDBC_E_INVALID, "null output");
    if (C < 4 || C > 64) return fail(VDBC_E_INVALID, "macrocell must be in [4, 64]");
    MediumK m;
    if ((s = make_medium(med, v.nx, v.ny, v.nz, &m))) return s;
    return launch_majorant<VdbAcc>(v, m, C, out, static_cast<hipStream_t>(stream));
}

extern "C" vdbc_status vdbc_majorant_dense(const float* dense, vdbc_dims d, float background,
                                           const vdbc_medium* med, uint32_t C, float* out,
                                           void* stream)
{
    clear_error();
    DenseView v;
    vdbc_status s = make_dense(dense, d, background, &v);
    if (s) return s;
    if (!out) return fail(VDBC_E_INVALID, "null output");
    if (C < 4 || C > 64) return fail(VDBC_E_INVALID, "macrocell must be in [4, 64]");
    MediumK m;
    if ((s = make_medium(med, v.nx, v.ny, v.nz, &m))) return s;
    return launch_majorant<DenseAcc>(v, m, C, out, static_cast<hipStream_t>(stream));
}

extern "C" vdbc_status vdbc_philox(const uint32_t* ctr, const uint32_t* key, uint64_t n,
                                   uint32_t* out, void* stream)
{
    clear_error();
    if (n && (!ctr || !key || !out)) return fail(VDBC_E_INVALID, "null argument");
    if (n > (uint64_t)0x7FFFFFFFull * kBlock) return fail(VDBC_E_INVALID, "too many counters");
    if (n == 0) return VDBC_OK;
    hipLaunchKernelGGL(philox_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       static_cast<hipStream_t>(stream), ctr, key, n, out);
    return launch_check("vdbc_philox");
}

// ---------------------------------------------------------------- batched PT (host)

struct vdbc_batch {
    uint32_t n = 0;
    vdbc_tuning t{};
    std::vector<VdbView> views;
    std::vector<CameraK> cams;
    std::vector<MediumK> meds;
    std::vector<PtArgs> gs;
    std::vector<float*> majs;
    std::vector<uint32_t*> coarse;
    std::vector<float*> images;
    std::vector<int> tiles_x, tiles_y;
    BatchDesc* d_descs = nullptr;
    uint32_t* d_items = nullptr;
    uint32_t* d_counter = nullptr;
    uint32_t n_items = 0;
    int max_cwords = 0;
    int grid_blocks = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace vdbc {

static vdbc_status batch_tuning(const vdbc_tuning* t, vdbc_tuning* out)
{
    vdbc_tuning d{16, 8, 4, 1};
    if (t) d = *t;
    if (d.macrocell < 4 || d.macrocell > 64 || (d.macrocell & (d.macrocell - 1)))
        return fail(VDBC_E_INVALID, "tuning.macrocell must be 4, 8, 16, 32 or 64");
    if (d.tile_w == 0) d.tile_w = 8;
    if (d.tile_w != 8 && d.tile_w != 16 && d.tile_w != 32 && d.tile_w != 64)
        return fail(VDBC_E_INVALID, "tuning.tile_w must be 8, 16, 32 or 64");
    if (d.blocks_per_cu == 0) d.blocks_per_cu = 4;
    if (d.blocks_per_cu > 32) return fail(VDBC_E_INVALID, "tuning.blocks_per_cu must be <= 32");
    *out = d;
    return VDBC_OK;
}

// Validates the items and fills the per-volume launch state; `layout`
// receives the workspace offsets (counter, descriptors, item list, then per
// volume majorant and coarse bits) and the total size.
static vdbc_status batch_plan(const vdbc_batch_item* items, uint32_t n, const vdbc_tuning& t, vdbc_batch* b,
                              std::vector<uint64_t>* maj_off, std::vector<uint64_t>* coarse_off,
                              uint64_t* items_off, uint64_t* total)
{
    if (!items || n == 0 || n > 4096) return fail(VDBC_E_INVALID, "need 1..4096 batch items");
    b->n = n;
    b->t = t;
    uint64_t tiles_total = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const vdbc_batch_item& it = items[i];
        VdbView v;
        CameraK cam;
        MediumK m;
        vdbc_status s = make_view(&it.grid, &v);
        if (!s) s = make_camera(&it.camera, &cam);
        if (!s) s = make_medium(&it.medium, v.nx, v.ny, v.nz, &m);
        if (s) return fail(s, "batch item %u: %s", i, vdbc_last_error());
        if (it.spp == 0 || it.max_bounces == 0 || !it.image)
            return fail(VDBC_E_INVALID, "batch item %u: spp, max_bounces >= 1 and an image are required", i);
        const double l = std::sqrt((double)it.medium.light_dir[0] * it.medium.light_dir[0] +
                                   (double)it.medium.light_dir[1] * it.medium.light_dir[1] +
                                   (double)it.medium.light_dir[2] * it.medium.light_dir[2]);
        if (!(std::fabs(l - 1.0) <= 1e-3)) return fail(VDBC_E_INVALID, "batch item %u: light_dir not unit", i);
        PtArgs g;
        pt_geometry(t.macrocell, v.nx, v.ny, v.nz, &g);
        g.spp = (int)it.spp;
        g.max_bounces = (int)it.max_bounces;
        g.tw = (int)t.tile_w;
        g.seed_lo = (uint32_t)it.seed;
        g.seed_hi = (uint32_t)(it.seed >> 32);
        g.frame = it.frame;
        g.rr = 0;
        const int tx = (cam.width + 2 * g.tw - 1) / (2 * g.tw), ty = (cam.height + 128 / g.tw - 1) / (128 / g.tw);
        if ((uint64_t)tx * ty > 0xFFFFFu) return fail(VDBC_E_INVALID, "batch item %u: image too large", i);
        b->views.push_back(v);
        b->cams.push_back(cam);
        b->meds.push_back(m);
        b->gs.push_back(g);
        b->images.push_back(it.image);
        b->tiles_x.push_back(tx);
        b->tiles_y.push_back(ty);
        tiles_total += (uint64_t)tx * ty;
        b->max_cwords = std::max(b->max_cwords, g.cwords);
    }
    uint64_t o = 256;                                   // counter
    const uint64_t descs_off = o;
    o += align256((uint64_t)n * sizeof(BatchDesc));
    *items_off = o;
    o += align256(tiles_total * 4);
    for (uint32_t i = 0; i < n; ++i) {
        maj_off->push_back(o);
        o += align256(majorant_bytes(t.macrocell, b->views[i].nx, b->views[i].ny, b->views[i].nz));
        coarse_off->push_back(o);
        o += align256(4ull * b->gs[i].cwords);
    }
    (void)descs_off;
    b->n_items = (uint32_t)tiles_total;
    *total = o;
    return VDBC_OK;
}

static vdbc_status batch_enqueue(vdbc_batch* b, hipStream_t st)
{
    vdbc_status s;
    for (uint32_t i = 0; i < b->n; ++i) {
        if ((s = launch_majorant<VdbAcc>(b->views[i], b->meds[i], (uint32_t)b->gs[i].C, b->majs[i], st))) return s;
        const PtArgs& g = b->gs[i];
        const uint64_t ncoarse = (uint64_t)g.cgx * g.cgy * g.cgz;
        hipLaunchKernelGGL(coarse_bits_kernel, dim3((unsigned)((ncoarse + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                           st, b->majs[i], g, b->coarse[i]);
        if ((s = launch_check("batch coarse occupancy"))) return s;
    }
    if (b->t.persistent) {
        hipLaunchKernelGGL(zero_u32, dim3(1), dim3(64), 0, st, b->d_counter);
        hipLaunchKernelGGL(pt_batch_kernel, dim3(b->grid_blocks), dim3(kBlock), 4u * (size_t)b->max_cwords, st,
                           b->d_descs, b->d_items, b->n_items, b->d_counter);
        return launch_check("batched render");
    }
    // one launch per volume; the launches run in stream order, so they share
    // the tile queue, cleared before each
    for (uint32_t i = 0; i < b->n; ++i) {
        const PtArgs& g = b->gs[i];
        const uint32_t tiles = (uint32_t)(b->tiles_x[i] * b->tiles_y[i]);
        hipLaunchKernelGGL(zero_u32, dim3(1), dim3(64), 0, st, b->d_counter);
        hipLaunchKernelGGL((pt_kernel<VdbAcc, VdbView, false, false>),
                           dim3(std::min<uint32_t>(tiles, (uint32_t)b->grid_blocks)), dim3(kBlock),
                           4u * (size_t)g.cwords, st, b->views[i], b->cams[i], b->meds[i], g, b->majs[i],
                           b->coarse[i], b->images[i], nullptr, nullptr, b->d_counter);
        if ((s = launch_check("per-volume render"))) return s;
    }
    return VDBC_OK;
}

}  // namespace vdbc

extern "C" vdbc_status vdbc_batch_workspace(const vdbc_batch_item* items, uint32_t n, const vdbc_tuning* t,
                                            uint64_t* bytes)
{
    clear_error();
    if (!bytes) return fail(VDBC_E_INVALID, "null argument");
    vdbc_tuning tt;
    vdbc_status s = batch_tuning(t, &tt);
    if (s) return s;
    vdbc_batch b;
    std::vector<uint64_t> mo, co;
    uint64_t io, total;
    if ((s = batch_plan(items, n, tt, &b, &mo, &co, &io, &total))) return s;
    *bytes = total;
    return VDBC_OK;
}

extern "C" vdbc_status vdbc_batch_create(const vdbc_batch_item* items, uint32_t n, const vdbc_tuning* t, void* ws,
                                         uint64_t ws_bytes, void* stream, vdbc_batch** out)
{
    clear_error();
    if (!out || !ws) return fail(VDBC_E_INVALID, "null argument");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(VDBC_E_INVALID, "workspace must be 256-byte aligned");
    *out = nullptr;
    vdbc_tuning tt;
    vdbc_status s = batch_tuning(t, &tt);
    if (s) return s;
    std::unique_ptr<vdbc_batch> b(new (std::nothrow) vdbc_batch());
    if (!b) return fail(VDBC_E_NOMEM, "no memory");
    std::vector<uint64_t> mo, co;
    uint64_t io, total;
    if ((s = batch_plan(items, n, tt, b.get(), &mo, &co, &io, &total))) return s;
    if (ws_bytes < total)
        return fail(VDBC_E_BUFFER_TOO_SMALL, "batch workspace needs %llu bytes", (unsigned long long)total);
    uint8_t* w = static_cast<uint8_t*>(ws);
    b->d_counter = reinterpret_cast<uint32_t*>(w);
    b->d_descs = reinterpret_cast<BatchDesc*>(w + 256);
    b->d_items = reinterpret_cast<uint32_t*>(w + io);
    for (uint32_t i = 0; i < n; ++i) {
        b->majs.push_back(reinterpret_cast<float*>(w + mo[i]));
        b->coarse.push_back(reinterpret_cast<uint32_t*>(w + co[i]));
    }
    // descriptors and the cost-ordered work list (largest estimated cost first:
    // samples per pixel x ray length through the volume)
    std::vector<BatchDesc> descs(n);
    std::vector<uint32_t> order(n);
    for (uint32_t i = 0; i < n; ++i) {
        descs[i] = BatchDesc{b->views[i], b->cams[i], b->meds[i], b->gs[i], b->majs[i], b->coarse[i], b->images[i],
                             b->tiles_x[i]};
        order[i] = i;
    }
    auto cost = [&](uint32_t i) {
        return (double)b->gs[i].spp * (double)(b->views[i].nx + b->views[i].ny + b->views[i].nz);
    };
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t c) { return cost(a) > cost(c); });
    std::vector<uint32_t> list;
    list.reserve(b->n_items);
    for (uint32_t i : order)
        for (uint32_t tl = 0; tl < (uint32_t)(b->tiles_x[i] * b->tiles_y[i]); ++tl) list.push_back((i << 20) | tl);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(b->d_descs, descs.data(), n * sizeof(BatchDesc), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(b->d_items, list.data(), list.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(VDBC_E_DEVICE, "batch descriptor upload: %s", hipGetErrorString(hipGetLastError()));
    b->grid_blocks = device_cus() * (int)tt.blocks_per_cu;
    *out = b.release();
    return VDBC_OK;
}

extern "C" vdbc_status vdbc_batch_launch(vdbc_batch* b, void* stream)
{
    clear_error();
    if (!b) return fail(VDBC_E_INVALID, "null batch");
    return batch_enqueue(b, static_cast<hipStream_t>(stream));
}

extern "C" vdbc_status vdbc_batch_capture(vdbc_batch* b, void* stream)
{
    clear_error();
    if (!b) return fail(VDBC_E_INVALID, "null batch");
    if (!stream) return fail(VDBC_E_INVALID, "capture needs a non-default stream");
    if (b->exec) return VDBC_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(VDBC_E_DEVICE, "begin capture: %s", hipGetErrorString(hipGetLastError()));
    vdbc_status s = batch_enqueue(b, st);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (s) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess || !g) return fail(VDBC_E_DEVICE, "end capture: %s", hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(VDBC_E_DEVICE, "graph instantiate failed");
    }
    b->graph = g;
    b->exec = ex;
    return VDBC_OK;
}

extern "C" vdbc_status vdbc_batch_graph_launch(vdbc_batch* b, void* stream)
{
    clear_error();
    if (!b || !b->exec) return fail(VDBC_E_INVALID, "batch has no captured graph");
    if (hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)) != hipSuccess)
        return fail(VDBC_E_DEVICE, "graph launch: %s", hipGetErrorString(hipGetLastError()));
    return VDBC_OK;
}

extern "C" void vdbc_batch_destroy(vdbc_batch* b)
{
    if (!b) return;
    // teardown: nothing useful can be done with a failure here
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    delete b;
}
