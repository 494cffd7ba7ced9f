// Shared by the HIP translation units: launch constants, device helpers for
// pixel tiles and block counters, and the host-side argument checks every
// launcher uses.
#pragma once
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

// ---------------------------------------------------------------- host helpers

static inline vdbc_status launch_check(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VDBC_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
    return VDBC_OK;
}

static inline vdbc_status make_view(const vdbc_grid* g, VdbView* v)
{
    if (!g || !g->device) return fail(VDBC_E_INVALID, "null grid");
    Header h;
    vdbc_status s = parse_header(g->header, g->bytes, &h);
    if (s) return s;
    if (h.layout != 0) return fail(VDBC_E_UNSUPPORTED, "the device kernels read node layout 0 only");
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

static inline vdbc_status make_dense(const float* dense, vdbc_dims d, float background, DenseView* v)
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

}  // namespace vdbc
