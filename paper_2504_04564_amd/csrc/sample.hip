// HIP kernels for gfx950 and their C-ABI launchers: random-access sampling of
// the compressed VDB and of the dense baseline (Section 3.2.2), integer
// lookups, the compression-error statistics of Section 5.2, and Philox words.
#include "kcommon.h"

namespace vdbc {

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

static vdbc_status check_samples(const float* pos, uint64_t n, uint32_t filter, float* out)
{
    if (filter > 1) return fail(VDBC_E_INVALID, "filter must be 0 or 1");
    if (n && (!pos || !out)) return fail(VDBC_E_INVALID, "null positions or output");
    if (n > (uint64_t)0x7FFFFFFFull * kBlock) return fail(VDBC_E_INVALID, "too many samples");
    return VDBC_OK;
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
