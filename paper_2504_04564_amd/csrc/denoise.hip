// Learned denoiser on gfx950: implicit-GEMM 3x3 convolutions (forward, data
// gradient, weight gradient) on v_mfma_f32_16x16x32_bf16 with FP32
// accumulation, the relative-MSE loss, ReLU/upsample backward, and Adam with
// FP32 master weights and BF16 copies.
//
// MFMA 16x16x32 BF16 operand layout (lane l, g = l / 16, r = l % 16):
// A[r][8g + j] and B[8g + j][r] for j < 8; the accumulator holds
// D[4g + i][r] for i < 4.  Every GEMM below puts its contraction index on K
// in chunks of 32 so that a lane's 8 K values are 8 consecutive channels of
// one 3x3 tap: one 16-byte load from an NHWC tensor.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "common.h"
#include "format.h"
#include "nn.h"

namespace vdbc {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kWgradChunkMax = 2048;   // output pixels per weight-gradient partial, at most
constexpr int kWgradChunkMin = 256;    // ... and at least
constexpr uint64_t kWgradGroups = 2048;   // workgroups a weight-gradient launch aims for (8 per CU)
constexpr int kConvTiles = 4;       // 16-pixel tiles per wave in the forward and data-gradient kernels
constexpr int kWgradStage = 64;     // output pixels staged in LDS per step of the weight-gradient kernel

// Output pixels per weight-gradient partial for P output pixels and a
// contraction of K: halved from the maximum while the launch (partials x
// 64-wide k tiles) would have fewer than kWgradGroups workgroups, so that
// the half-resolution layers and the narrow first layer fill the chip.
int wgrad_chunk(uint64_t P, int K)
{
    const uint64_t kb = (uint64_t)(K + 63) / 64;
    int c = kWgradChunkMax;
    while (c > kWgradChunkMin && (P + c - 1) / c * kb < kWgradGroups) c /= 2;
    return c;
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ bf16x8 load8(const uint16_t* p)
{
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}
__device__ __forceinline__ bf16x8 zero8() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }
__device__ __forceinline__ f4 mfma(bf16x8 a, bf16x8 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Input of a convolution: channels [0, ca) from `a`, [ca, ca + cb) from `b`
// (a channel concat), both NHWC of spatial size hs x ws; with `up` they are
// read through a nearest-neighbour x2 upsample.
struct ConvIn {
    const uint16_t* a;
    const uint16_t* b;
    int ca, cb, up, n, hs, ws;
};

__device__ __forceinline__ bf16x8 gather8(const ConvIn& in, int n, int iy, int ix, int c0)
{
    const int hv = in.up ? 2 * in.hs : in.hs, wv = in.up ? 2 * in.ws : in.ws;
    if ((unsigned)iy >= (unsigned)hv || (unsigned)ix >= (unsigned)wv) return zero8();
    const int sy = in.up ? iy >> 1 : iy, sx = in.up ? ix >> 1 : ix;
    const int64_t pix = ((int64_t)n * in.hs + sy) * in.ws + sx;
    return c0 < in.ca ? load8(in.a + pix * in.ca + c0) : load8(in.b + pix * in.cb + (c0 - in.ca));
}

// ---------------------------------------------------------------- forward
// out[p][co] = act(bias[co] + sum_k A[p][k] W[co][k]), k = tap * cin + ci.
// A wave computes MB tiles of 16 output pixels x NT tiles of 16 channels
// (64 MB pixels per workgroup): each weight fragment it loads feeds MB MFMAs.
template <int NT, int MB>
__global__ __launch_bounds__(kThreads) void conv_fwd_kernel(ConvIn in, const uint16_t* __restrict__ w,
                                                            const float* __restrict__ bias, int cout,
                                                            int stride, int ho, int wo, int relu,
                                                            uint16_t* __restrict__ out_bf,
                                                            float* __restrict__ out_f,
                                                            const uint16_t* __restrict__ resid)
{
    const int cin = in.ca + in.cb, K = 9 * cin;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
    const int64_t P = (int64_t)in.n * ho * wo;
    const int64_t p0 = ((int64_t)blockIdx.x * 4 + wave) * 16 * MB;   // first pixel of the wave
    bool pv[MB];
    int n[MB], oy[MB], ox[MB];
#pragma unroll
    for (int m = 0; m < MB; ++m) {
        const int64_t p = p0 + 16 * m + r;
        pv[m] = p < P;
        const int64_t pc = pv[m] ? p : 0;
        ox[m] = (int)(pc % wo);
        const int64_t q = pc / wo;
        oy[m] = (int)(q % ho);
        n[m] = (int)(q / ho);
    }
    f4 acc[MB][NT];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    // operands of k step kb + 32 are loaded while the MFMAs of step kb run
    bf16x8 Bn[NT], An[MB];
    auto fetch = [&](int kb) {
        const int k = kb + 8 * g;
        const int tap = k / cin, c0 = k - tap * cin;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int co = t * 16 + r;
            Bn[t] = (co < cout && tap < 9) ? load8(w + (int64_t)co * K + k) : zero8();
        }
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            An[m] = zero8();
            if (pv[m] && tap < 9)
                An[m] = gather8(in, n[m], oy[m] * stride + tap / 3 - 1, ox[m] * stride + tap % 3 - 1, c0);
        }
    };
    fetch(0);
    for (int kb = 0; kb < K; kb += 32) {
        bf16x8 B[NT], A[MB];
#pragma unroll
        for (int t = 0; t < NT; ++t) B[t] = Bn[t];
#pragma unroll
        for (int m = 0; m < MB; ++m) A[m] = An[m];
        if (kb + 32 < K) fetch(kb + 32);
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[m][t] = mfma(A[m], B[t], acc[m][t]);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int co = t * 16 + r;
        if (co >= cout) continue;
        const float bb = bias[co];
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t pp = p0 + 16 * m + 4 * g + i;
                if (pp >= P) continue;
                float v = acc[m][t][i] + bb;
                if (relu) v = fmaxf(v, 0.0f);
                if (out_f) {
                    if (resid) v += bf2f(resid[pp * 8 + co]);
                    out_f[pp * cout + co] = v;
                } else {
                    out_bf[pp * cout + co] = f2bf(v);
                }
            }
    }
}

// Stride-1 forward on a two-dimensional output tile: the workgroup stages
// its input tile (kFwdTH + 2) x (kFwdTW + 2) pixels x cin channels once in
// LDS (zero outside the image; through the upsample / concat of ConvIn), so
// the nine taps read shifted views of it instead of gathering every input
// pixel from memory once per tap.  Pixels are padded by one 16-byte group in
// LDS so that the 16 lanes of an operand fetch, reading consecutive pixels,
// spread over the banks.  Wave w computes output rows 2w and 2w + 1, each
// as two 16-pixel tiles, times NT tiles of 16 channels.
constexpr int kFwdTH = 8, kFwdTW = 32;
constexpr int kEpiStride = kFwdTH * kFwdTW + 4;   // channel stride of an epilogue staged through LDS

// Forward epilogue through LDS (BF16 output, cout a multiple of 4): the
// accumulators go to LDS channel-major as in the data gradient's staged
// epilogue, 32 channels per pass; then each thread takes four channels of
// one pixel, adds the bias, applies the ReLU and writes the four BF16 values
// as one 8-byte store.  Per element the arithmetic is the direct epilogue's.
template <int NT>
__device__ __forceinline__ void fwd_store_staged(float* s_out, const f4 (&acc)[4][NT], const int (&run_pix)[4],
                                                 const float* __restrict__ bias, int cout, int relu, int ty0,
                                                 int tx0, int n, int ho, int wo, uint16_t* __restrict__ out_bf)
{
    constexpr int PT = NT < 2 ? NT : 2;
    const int r = threadIdx.x & 15;
#pragma unroll
    for (int pass = 0; pass < NT / PT; ++pass) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int tt = 0; tt < PT; ++tt) {
                const f4 a = acc[k][pass * PT + tt];
                *reinterpret_cast<float4*>(s_out + (tt * 16 + r) * kEpiStride + run_pix[k]) =
                    make_float4(a[0], a[1], a[2], a[3]);
            }
        __syncthreads();
        const int c_lo = pass * PT * 16, c_hi = min(cout, c_lo + PT * 16);
        const int groups = (c_hi - c_lo) / 4;
        for (int e = threadIdx.x; e < kFwdTH * kFwdTW * groups; e += kThreads) {
            const int p = e / groups, c = c_lo + (e - p * groups) * 4;
            const int y = ty0 + p / kFwdTW, x = tx0 + p % kFwdTW;
            if (y >= ho || x >= wo) continue;
            const int64_t pp = ((int64_t)n * ho + y) * wo + x;
            uint16_t out[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float v = s_out[(c - c_lo + j) * kEpiStride + p] + bias[c + j];
                if (relu) v = fmaxf(v, 0.0f);
                out[j] = f2bf(v);
            }
            *reinterpret_cast<uint2*>(out_bf + pp * cout + c) =
                make_uint2((uint32_t)out[0] | (uint32_t)out[1] << 16, (uint32_t)out[2] | (uint32_t)out[3] << 16);
        }
    }
}

template <int NT, bool STAGED>
__global__ __launch_bounds__(kThreads) void conv_fwd_tiled_kernel(ConvIn in, const uint16_t* __restrict__ w,
                                                                  const float* __restrict__ bias, int cout,
                                                                  int ho, int wo, int relu,
                                                                  uint16_t* __restrict__ out_bf,
                                                                  float* __restrict__ out_f,
                                                                  const uint16_t* __restrict__ resid)
{
    extern __shared__ uint4 s_tile[];
    const int cin = in.ca + in.cb, K = 9 * cin, cg = cin / 8, ps = cg + 1;
    constexpr int IW = kFwdTW + 2, IH = kFwdTH + 2;
    const int tx0 = blockIdx.x * kFwdTW, ty0 = blockIdx.y * kFwdTH, n = blockIdx.z;
    for (int e = threadIdx.x; e < IH * IW * cg; e += kThreads) {
        const int pix = e / cg, c8 = e - pix * cg;
        const int iy = ty0 - 1 + pix / IW, ix = tx0 - 1 + pix % IW;
        s_tile[pix * ps + c8] = __builtin_bit_cast(uint4, gather8(in, n, iy, ix, 8 * c8));
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
    f4 acc[4][NT];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int kb = 0; kb < K; kb += 32) {
        const int k = kb + 8 * g;
        const int tap = k / cin, c0 = k - tap * cin;
        const bool valid = tap < 9;
        const int ky = tap / 3, kx = tap - 3 * (tap / 3);
        bf16x8 B[NT], A[4];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int co = t * 16 + r;
            B[t] = (co < cout && valid) ? load8(w + (int64_t)co * K + k) : zero8();
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int row = 2 * wave + (m >> 1) + ky, col = (m & 1) * 16 + r + kx;
            A[m] = valid ? __builtin_bit_cast(bf16x8, s_tile[(row * IW + col) * ps + c0 / 8]) : zero8();
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[m][t] = mfma(A[m], B[t], acc[m][t]);
    }
    if constexpr (STAGED) {
        // tile m holds pixels (m & 1) * 16 + 4g .. + 3 of row 2w + (m >> 1)
        int run_pix[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) run_pix[m] = (2 * wave + (m >> 1)) * kFwdTW + (m & 1) * 16 + 4 * g;
        fwd_store_staged<NT>(reinterpret_cast<float*>(s_tile), acc, run_pix, bias, cout, relu, ty0, tx0, n, ho, wo,
                             out_bf);
        return;
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int co = t * 16 + r;
        if (co >= cout) continue;
        const float bb = bias[co];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int y = ty0 + 2 * wave + (m >> 1);
            if (y >= ho) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = tx0 + (m & 1) * 16 + 4 * g + i;
                if (x >= wo) continue;
                const int64_t pp = ((int64_t)n * ho + y) * wo + x;
                float v = acc[m][t][i] + bb;
                if (relu) v = fmaxf(v, 0.0f);
                if (out_f) {
                    if (resid) v += bf2f(resid[pp * 8 + co]);
                    out_f[pp * cout + co] = v;
                } else {
                    out_bf[pp * cout + co] = f2bf(v);
                }
            }
        }
    }
}

// ---------------------------------------------------------------- data gradient
// dx[q][c] (+)= sum_{tap, co} dz[p(q, tap)][co] Wt[c][tap][co] over the input
// pixels q of the (virtual) input; p = ((y+1-ky)/s, (x+1-kx)/s) when that is
// an integer output position.  dz has channel stride coutp (multiple of 8),
// Wt is the transposed weight [cin][9][coutp].  A wave computes MB tiles of
// 16 input pixels x NT tiles of 16 channels, as the forward kernel.
// Where the data gradient goes.  Channels [0, split) are written (or added,
// with `accumulate`) as FP32 to dx with dx_stride channels per pixel.
// Channels [split, cin) are the backward of the ReLU that produced the
// layer's input: dz[q][c - split] = BF16((dx + add) * (y > 0)), with `add`
// an optional FP32 gradient of the same activation from another branch;
// this is the whole input of the next layer's backward, so no FP32 copy of
// those channels is written.
struct DgradOut {
    float* dx;
    int dx_stride, accumulate, split;
    uint16_t* dz;
    int dz_stride;
    const uint16_t* y;
    int y_stride;
    const float* add;
    int add_stride;
    // The layer's input was upsampled x2 from the activation y: each 2 x 2
    // block of the data gradient is summed (the upsample's backward) before
    // the ReLU backward, and dz is written at half resolution (split 0,
    // stride-1 tiled kernel only).
    int pool;
    // Set by the launcher: every pointer above aligned for 16-byte (FP32)
    // and 8-byte (BF16) accesses of four channels, strides multiples of 4.
    int vec;
};

template <int NT, int MB>
__global__ __launch_bounds__(kThreads) void conv_dgrad_kernel(const uint16_t* __restrict__ dz, int coutp,
                                                              int n_img, int ho, int wo,
                                                              const uint16_t* __restrict__ wt, int cin,
                                                              int stride, int hv, int wv, DgradOut o)
{
    const int K = 9 * coutp;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
    const int64_t Q = (int64_t)n_img * hv * wv;
    const int64_t q0 = ((int64_t)blockIdx.x * 4 + wave) * 16 * MB;   // first pixel of the wave
    bool qv[MB];
    int n[MB], iy[MB], ix[MB];
#pragma unroll
    for (int m = 0; m < MB; ++m) {
        const int64_t q = q0 + 16 * m + r;
        qv[m] = q < Q;
        const int64_t qc = qv[m] ? q : 0;
        ix[m] = (int)(qc % wv);
        const int64_t t = qc / wv;
        iy[m] = (int)(t % hv);
        n[m] = (int)(t / hv);
    }
    f4 acc[MB][NT];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int kb = 0; kb < K; kb += 32) {
        const int k = kb + 8 * g;
        const int tap = k / coutp, co0 = k - tap * coutp;
        bf16x8 B[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = t * 16 + r;
            B[t] = (c < cin && tap < 9) ? load8(wt + (int64_t)c * K + k) : zero8();
        }
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            bf16x8 A = zero8();
            if (qv[m] && tap < 9) {
                const int ty = iy[m] + 1 - tap / 3, tx = ix[m] + 1 - tap % 3;
                if (ty >= 0 && tx >= 0 && ty % stride == 0 && tx % stride == 0) {
                    const int oy = ty / stride, ox = tx / stride;
                    if (oy < ho && ox < wo) A = load8(dz + (((int64_t)n[m] * ho + oy) * wo + ox) * coutp + co0);
                }
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[m][t] = mfma(A, B[t], acc[m][t]);
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int c = t * 16 + r;
        if (c >= cin) continue;
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t qq = q0 + 16 * m + 4 * g + i;
                if (qq >= Q) continue;
                float v = acc[m][t][i];
                if (c < o.split) {
                    float* d = o.dx + qq * o.dx_stride + c;
                    *d = o.accumulate ? *d + v : v;
                } else {
                    const int cc = c - o.split;
                    if (o.add) v += o.add[qq * o.add_stride + cc];
                    if (!(bf2f(o.y[qq * o.y_stride + cc]) > 0.0f)) v = 0.0f;
                    o.dz[qq * o.dz_stride + cc] = f2bf(v);
                }
            }
    }
}

// Epilogue of a data-gradient kernel through LDS.  The accumulators of the
// workgroup's kFwdTH x kFwdTW pixel tile go to LDS channel-major, FP32
// [channel][pixel] with a channel stride of 256 + 4 floats, 32 channels per
// pass: a lane holds
// one channel of several pixels, and the caller passes them as 16-byte runs
// of consecutive pixels (runs[n] holds pixels run_pix[n] .. + 3 of channel
// t * 16 + r for run n of channel tile t).  Then each thread takes four
// channels of one pixel at a time, so that neighbouring threads read and
// write neighbouring 16-byte (FP32) and 8-byte (BF16) pieces of memory.  Per
// element the arithmetic is that of the direct epilogue.
// Channels [c_lo, c_hi) of the tile, staged channel-major from channel c_lo.
__device__ __forceinline__ void dgrad_store_pass(const float* s_out, int c_lo, int c_hi, int ty0, int tx0, int n,
                                                 int hv, int wv, const DgradOut& o)
{
    const int groups = (c_hi - c_lo) / 4;
    for (int e = threadIdx.x; e < kFwdTH * kFwdTW * groups; e += kThreads) {
        const int p = e / groups, c = c_lo + (e - p * groups) * 4;
        const int y = ty0 + p / kFwdTW, x = tx0 + p % kFwdTW;
        if (y >= hv || x >= wv) continue;
        const int64_t qq = ((int64_t)n * hv + y) * wv + x;
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = s_out[(c - c_lo + j) * kEpiStride + p];
        if (c < o.split) {
            float* d = o.dx + qq * o.dx_stride + c;
            if (o.vec) {
                float4* d4 = reinterpret_cast<float4*>(d);
                if (o.accumulate) {
                    const float4 b = *d4;
                    v[0] = b.x + v[0];
                    v[1] = b.y + v[1];
                    v[2] = b.z + v[2];
                    v[3] = b.w + v[3];
                }
                *d4 = make_float4(v[0], v[1], v[2], v[3]);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) d[j] = o.accumulate ? d[j] + v[j] : v[j];
            }
        } else {
            const int cc = c - o.split;
            const uint16_t* yp = o.y + qq * o.y_stride + cc;
            uint16_t* zp = o.dz + qq * o.dz_stride + cc;
            uint16_t yv[4], out[4];
            if (o.vec) {
                if (o.add) {
                    const float4 b = *reinterpret_cast<const float4*>(o.add + qq * o.add_stride + cc);
                    v[0] += b.x;
                    v[1] += b.y;
                    v[2] += b.z;
                    v[3] += b.w;
                }
                const uint2 yy = *reinterpret_cast<const uint2*>(yp);
                yv[0] = (uint16_t)(yy.x & 0xFFFFu);
                yv[1] = (uint16_t)(yy.x >> 16);
                yv[2] = (uint16_t)(yy.y & 0xFFFFu);
                yv[3] = (uint16_t)(yy.y >> 16);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (o.add) v[j] += o.add[qq * o.add_stride + cc + j];
                    yv[j] = yp[j];
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) out[j] = f2bf(bf2f(yv[j]) > 0.0f ? v[j] : 0.0f);
            if (o.vec) {
                *reinterpret_cast<uint2*>(zp) =
                    make_uint2((uint32_t)out[0] | (uint32_t)out[1] << 16, (uint32_t)out[2] | (uint32_t)out[3] << 16);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) zp[j] = out[j];
            }
        }
    }
}

template <int NT>
__device__ __forceinline__ void dgrad_store_staged(float* s_out, const float4 (&runs)[4][NT], const int (&run_pix)[4],
                                                   int cin, int ty0, int tx0, int n, int hv, int wv,
                                                   const DgradOut& o)
{
    // at most two channel tiles (32 channels) per pass, so that the buffer
    // stays at 33 KB and more workgroups fit on a CU
    constexpr int PT = NT < 2 ? NT : 2;
    const int r = threadIdx.x & 15;
#pragma unroll
    for (int pass = 0; pass < NT / PT; ++pass) {
        __syncthreads();   // the staged window, or the previous pass, is done with
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int tt = 0; tt < PT; ++tt)
                *reinterpret_cast<float4*>(s_out + (tt * 16 + r) * kEpiStride + run_pix[k]) = runs[k][pass * PT + tt];
        __syncthreads();
        const int c_lo = pass * PT * 16, c_hi = min(cin, c_lo + PT * 16);
        if (c_lo < c_hi) dgrad_store_pass(s_out, c_lo, c_hi, ty0, tx0, n, hv, wv, o);
    }
}


// Stride-1 data gradient on a two-dimensional tile of input pixels, the
// forward tile scheme with the taps mirrored: the workgroup stages dz over
// its (kFwdTH + 2) x (kFwdTW + 2) window (zero outside the output) once in
// LDS, and tap (ky, kx) of input pixel (y, x) reads dz at (y + 1 - ky,
// x + 1 - kx), a shifted view of the window.  Same contraction order,
// operands and epilogue as conv_dgrad_kernel.
template <int NT, bool STAGED>
__global__ __launch_bounds__(kThreads) void conv_dgrad_tiled_kernel(const uint16_t* __restrict__ dz, int coutp,
                                                                    int ho, int wo,
                                                                    const uint16_t* __restrict__ wt, int cin,
                                                                    DgradOut o)
{
    extern __shared__ uint4 s_tile[];
    const int K = 9 * coutp, cg = coutp / 8, ps = cg + 1;
    constexpr int IW = kFwdTW + 2, IH = kFwdTH + 2;
    const int tx0 = blockIdx.x * kFwdTW, ty0 = blockIdx.y * kFwdTH, n = blockIdx.z;
    for (int e = threadIdx.x; e < IH * IW * cg; e += kThreads) {
        const int pix = e / cg, c8 = e - pix * cg;
        const int y = ty0 - 1 + pix / IW, x = tx0 - 1 + pix % IW;
        uint4 v = make_uint4(0, 0, 0, 0);
        if ((unsigned)y < (unsigned)ho && (unsigned)x < (unsigned)wo)
            v = *reinterpret_cast<const uint4*>(dz + (((int64_t)n * ho + y) * wo + x) * coutp + 8 * c8);
        s_tile[pix * ps + c8] = v;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
    f4 acc[4][NT];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int kb = 0; kb < K; kb += 32) {
        const int k = kb + 8 * g;
        const int tap = k / coutp, co0 = k - tap * coutp;
        const bool valid = tap < 9;
        const int ky = tap / 3, kx = tap - 3 * (tap / 3);
        bf16x8 B[NT], A[4];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = t * 16 + r;
            B[t] = (c < cin && valid) ? load8(wt + (int64_t)c * K + k) : zero8();
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int row = 2 * wave + (m >> 1) + 2 - ky, col = (m & 1) * 16 + r + 2 - kx;
            A[m] = valid ? __builtin_bit_cast(bf16x8, s_tile[(row * IW + col) * ps + co0 / 8]) : zero8();
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[m][t] = mfma(A[m], B[t], acc[m][t]);
    }
    if constexpr (STAGED) {
        // tile m holds pixels (m & 1) * 16 + 4g .. + 3 of row 2w + (m >> 1)
        int run_pix[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) run_pix[m] = (2 * wave + (m >> 1)) * kFwdTW + (m & 1) * 16 + 4 * g;
        float4 runs[4][NT];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int t = 0; t < NT; ++t) runs[m][t] = make_float4(acc[m][t][0], acc[m][t][1], acc[m][t][2], acc[m][t][3]);
        dgrad_store_staged<NT>(reinterpret_cast<float*>(s_tile), runs, run_pix, cin, ty0, tx0, n, ho, wo, o);
        return;
    }
    if (o.pool) {
        // rows 2w and 2w + 1 of the tile are tiles m and m + 2; columns
        // 4g + i pair as (0, 1) and (2, 3) in one lane; ho and wo are even
        const int y2 = ty0 / 2 + wave, h2 = ho / 2, w2 = wo / 2;
        if (y2 >= h2) return;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = t * 16 + r;
            if (c >= cin) continue;
#pragma unroll
            for (int mc = 0; mc < 2; ++mc)
#pragma unroll
                for (int ip = 0; ip < 2; ++ip) {
                    const int x2 = (tx0 + mc * 16 + 4 * g) / 2 + ip;
                    if (x2 >= w2) continue;
                    const int64_t qh = ((int64_t)n * h2 + y2) * w2 + x2;
                    float v = ((acc[mc][t][2 * ip] + acc[mc][t][2 * ip + 1]) + acc[mc + 2][t][2 * ip]) +
                              acc[mc + 2][t][2 * ip + 1];
                    if (!(bf2f(o.y[qh * o.y_stride + c]) > 0.0f)) v = 0.0f;
                    o.dz[qh * o.dz_stride + c] = f2bf(v);
                }
        }
        return;
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int c = t * 16 + r;
        if (c >= cin) continue;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int y = ty0 + 2 * wave + (m >> 1);
            if (y >= ho) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = tx0 + (m & 1) * 16 + 4 * g + i;
                if (x >= wo) continue;
                const int64_t qq = ((int64_t)n * ho + y) * wo + x;
                float v = acc[m][t][i];
                if (c < o.split) {
                    float* d = o.dx + qq * o.dx_stride + c;
                    *d = o.accumulate ? *d + v : v;
                } else {
                    const int cc = c - o.split;
                    if (o.add) v += o.add[qq * o.add_stride + cc];
                    if (!(bf2f(o.y[qq * o.y_stride + cc]) > 0.0f)) v = 0.0f;
                    o.dz[qq * o.dz_stride + cc] = f2bf(v);
                }
            }
        }
    }
}

// Stride-2 data gradient by parity class: input pixel (y, x) takes tap
// (ky, kx) only where y + 1 - ky and x + 1 - kx are even, so rows of even y
// take ky = 1 alone and rows of odd y take ky = 0 and 2 (columns likewise):
// 9 of the 36 (class, tap) pairs of a 2 x 2 pixel block.  Wave w takes
// input rows ty0 + 2w (even) and ty0 + 2w + 1 (odd), each as a 16-pixel
// tile of even and one of odd columns, so every MFMA tile is one parity
// class and runs over its own taps only; the dz window under the
// kFwdTH x kFwdTW input tile, (kFwdTH / 2 + 1) x (kFwdTW / 2 + 1) output
// pixels, is staged in LDS once.  Chunks of 32 k (one tap, 32 output
// channels) are added in the order of conv_dgrad_kernel, which adds only
// zeros between them.
template <int NT>
__global__ __launch_bounds__(kThreads) void conv_dgrad_s2_kernel(const uint16_t* __restrict__ dz, int coutp,
                                                                 int ho, int wo,
                                                                 const uint16_t* __restrict__ wt, int cin,
                                                                 int hv, int wv, DgradOut o)
{
    extern __shared__ uint4 s_tile[];
    const int K = 9 * coutp, cg = coutp / 8, ps = cg + 1;
    constexpr int IW = kFwdTW / 2 + 1, IH = kFwdTH / 2 + 1;
    const int tx0 = blockIdx.x * kFwdTW, ty0 = blockIdx.y * kFwdTH, n = blockIdx.z;
    const int oy0 = ty0 / 2, ox0 = tx0 / 2;
    for (int e = threadIdx.x; e < IH * IW * cg; e += kThreads) {
        const int pix = e / cg, c8 = e - pix * cg;
        const int y = oy0 + pix / IW, x = ox0 + pix % IW;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (y < ho && x < wo)
            v = *reinterpret_cast<const uint4*>(dz + (((int64_t)n * ho + y) * wo + x) * coutp + 8 * c8);
        s_tile[pix * ps + c8] = v;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
    f4 acc[4][NT];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int py = m >> 1, px = m & 1;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int ky = tap / 3, kx = tap % 3;
            if (((py + 1 - ky) & 1) || ((px + 1 - kx) & 1)) continue;
            const int row = (2 * wave + py + 1 - ky) / 2, col = (2 * r + px + 1 - kx) / 2;
            for (int cc = 0; cc < coutp; cc += 32) {
                const int co0 = cc + 8 * g;
                const bool valid = co0 < coutp;
                const bf16x8 A = valid ? __builtin_bit_cast(bf16x8, s_tile[(row * IW + col) * ps + co0 / 8]) : zero8();
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const int c = t * 16 + r;
                    const bf16x8 B = (c < cin && valid) ? load8(wt + (int64_t)c * K + tap * coutp + co0) : zero8();
                    acc[m][t] = mfma(A, B, acc[m][t]);
                }
            }
        }
    }
    if constexpr (NT <= 2) {
        // row 2w + h holds pixels 8g .. 8g + 7 of this lane's channel as
        // tiles m = 2h (even columns) and 2h + 1 (odd columns), interleaved
        float4 runs[4][NT];
        int run_pix[4];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            run_pix[2 * h] = (2 * wave + h) * kFwdTW + 8 * g;
            run_pix[2 * h + 1] = run_pix[2 * h] + 4;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const f4 e = acc[2 * h][t], d = acc[2 * h + 1][t];
                runs[2 * h][t] = make_float4(e[0], d[0], e[1], d[1]);
                runs[2 * h + 1][t] = make_float4(e[2], d[2], e[3], d[3]);
            }
        }
        dgrad_store_staged<NT>(reinterpret_cast<float*>(s_tile), runs, run_pix, cin, ty0, tx0, n, hv, wv, o);
        return;
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int c = t * 16 + r;
        if (c >= cin) continue;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int y = ty0 + 2 * wave + (m >> 1);
            if (y >= hv) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = tx0 + 2 * (4 * g + i) + (m & 1);
                if (x >= wv) continue;
                const int64_t qq = ((int64_t)n * hv + y) * wv + x;
                float v = acc[m][t][i];
                if (c < o.split) {
                    float* d = o.dx + qq * o.dx_stride + c;
                    *d = o.accumulate ? *d + v : v;
                } else {
                    const int cc = c - o.split;
                    if (o.add) v += o.add[qq * o.add_stride + cc];
                    if (!(bf2f(o.y[qq * o.y_stride + cc]) > 0.0f)) v = 0.0f;
                    o.dz[qq * o.dz_stride + cc] = f2bf(v);
                }
            }
        }
    }
}

// Wt[c][tap][co] = W[co][tap][c] (zero for co >= cout), BF16.
__global__ void transpose_weights_kernel(const uint16_t* __restrict__ w, int cin, int cout, int coutp,
                                         uint16_t* __restrict__ wt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cin * 9 * coutp) return;
    const int co = i % coutp, tap = (i / coutp) % 9, c = i / (9 * coutp);
    wt[i] = co < cout ? w[((int64_t)co * 9 + tap) * cin + c] : (uint16_t)0;
}

// The transposes of up to five layers in one launch (a training step's data
// gradients): workgroup y takes layer y.
struct WtJobs {
    const uint16_t* w[5];
    uint16_t* wt[5];
    int cin[5], cout[5], coutp[5];
};

__global__ void transpose_weights_many_kernel(WtJobs j)
{
    const int l = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= j.cin[l] * 9 * j.coutp[l]) return;
    const int coutp = j.coutp[l], cin = j.cin[l];
    const int co = i % coutp, tap = (i / coutp) % 9, c = i / (9 * coutp);
    j.wt[l][i] = co < j.cout[l] ? j.w[l][((int64_t)co * 9 + tap) * cin + c] : (uint16_t)0;
}

// ---------------------------------------------------------------- weight gradient
// partial[chunk][co][k] = sum over the chunk's output pixels p of
// dz[p][co] * A[p][k] with A the forward operand (k = tap * cin + ci).
// M = co (MT tiles of 16), N = k (64 per workgroup, 16 per wave), K = pixels
// staged kWgradStage at a time through LDS (dz rows and im2col rows, both
// contiguous) and consumed 32 per MFMA in pixel order.
// The workgroups of the first k tile also sum the staged dz rows per channel:
// bpart[chunk][c] = sum over the chunk's pixels of dz[p][c] (thread (w, c)
// adds pixels w, w + 4, ... of each staged block, then the four wave sums in
// order), the bias gradient's partials.
template <int MT>
__global__ __launch_bounds__(kThreads) void conv_wgrad_kernel(ConvIn in, int stride, int ho, int wo,
                                                              const uint16_t* __restrict__ dz, int coutp, int chunk,
                                                              float* __restrict__ partial, float* __restrict__ bpart)
{
    __shared__ uint16_t sA[kWgradStage][64 + 8];
    __shared__ uint16_t sB[kWgradStage][64 + 8];
    const int cin = in.ca + in.cb, K = 9 * cin;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, r = lane & 15;
    const int kbase = blockIdx.y * 64;
    const int64_t P = (int64_t)in.n * ho * wo;
    const int64_t p0 = (int64_t)blockIdx.x * chunk;
    const int64_t p1 = p0 + chunk < P ? p0 + chunk : P;
    f4 acc[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) acc[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    const int cg = coutp / 8;
    const bool bias = blockIdx.y == 0;   // uniform per workgroup
    const bool small = P <= 0x7FFFFFFF;  // pixel indices fit 31 bits
    float bsum = 0.0f;
    // The global loads of the next stage are issued before the MFMAs of the
    // current one and land in registers; they are written to LDS at the top
    // of the next step, so each step waits on loads issued a step earlier.
    uint4 ra[kWgradStage * 8 / kThreads];   // dz rows: kWgradStage pixels x coutp (<= 64) channels
    uint4 rb[kWgradStage / 32];             // im2col rows: kWgradStage pixels x 64 values of k
    auto fetch = [&](int64_t pb) {
#pragma unroll
        for (int i = 0; i < kWgradStage * 8 / kThreads; ++i) {
            const int idx = tid + kThreads * i, px = idx / cg, c8 = (idx - px * cg) * 8;
            ra[i] = make_uint4(0, 0, 0, 0);
            if (idx < kWgradStage * cg && pb + px < p1)
                ra[i] = *reinterpret_cast<const uint4*>(dz + (pb + px) * coutp + c8);
        }
#pragma unroll
        for (int it = 0; it < kWgradStage / 32; ++it) {
            const int px = (tid >> 3) + 32 * it, kg = tid & 7;
            const int k = kbase + kg * 8;
            bf16x8 v = zero8();
            const int64_t p = pb + px;
            if (p < p1 && k < K) {
                const int tap = k / cin, c0 = k - tap * cin;
                int ox, oy, n;
                if (small) {   // 32-bit division (uniform branch)
                    const uint32_t pu = (uint32_t)p, q = pu / (uint32_t)wo, nn = q / (uint32_t)ho;
                    ox = (int)(pu - q * (uint32_t)wo);
                    oy = (int)(q - nn * (uint32_t)ho);
                    n = (int)nn;
                } else {
                    ox = (int)(p % wo);
                    const int64_t q = p / wo;
                    oy = (int)(q % ho);
                    n = (int)(q / ho);
                }
                v = gather8(in, n, oy * stride + tap / 3 - 1, ox * stride + tap % 3 - 1, c0);
            }
            rb[it] = __builtin_bit_cast(uint4, v);
        }
    };
    fetch(p0);
    for (int64_t pb = p0; pb < p1; pb += kWgradStage) {
#pragma unroll
        for (int i = 0; i < kWgradStage * 8 / kThreads; ++i) {
            const int idx = tid + kThreads * i, px = idx / cg, c8 = (idx - px * cg) * 8;
            if (idx < kWgradStage * cg) *reinterpret_cast<uint4*>(&sA[px][c8]) = ra[i];
        }
#pragma unroll
        for (int it = 0; it < kWgradStage / 32; ++it)
            *reinterpret_cast<uint4*>(&sB[(tid >> 3) + 32 * it][(tid & 7) * 8]) = rb[it];
        __syncthreads();
        if (pb + kWgradStage < p1) fetch(pb + kWgradStage);
        if (bias && lane < coutp) {
            // rows past the chunk's end were staged as zeros
#pragma unroll 8
            for (int j = 0; j < kWgradStage / 4; ++j) bsum += bf2f(sA[wave + 4 * j][lane]);
        }
#pragma unroll
        for (int sub = 0; sub < kWgradStage; sub += 32) {
            bf16x8 B;
#pragma unroll
            for (int j = 0; j < 8; ++j) B[j] = __builtin_bit_cast(__bf16, sB[sub + 8 * g + j][16 * wave + r]);
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                bf16x8 A;
                const int co = t * 16 + r;
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    A[j] = co < coutp ? __builtin_bit_cast(__bf16, sA[sub + 8 * g + j][co]) : (__bf16)0.0f;
                acc[t] = mfma(A, B, acc[t]);
            }
        }
        __syncthreads();
    }
    if (bias) {
        __shared__ float sred[4][64];
        sred[wave][lane] = bsum;
        __syncthreads();
        if (tid < coutp)
            bpart[(int64_t)blockIdx.x * coutp + tid] = ((sred[0][tid] + sred[1][tid]) + sred[2][tid]) + sred[3][tid];
    }
    const int k = kbase + 16 * wave + r;
    if (k >= K) return;
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int co = t * 16 + 4 * g + i;
            partial[((int64_t)blockIdx.x * (MT * 16) + co) * K + k] = acc[t][i];
        }
}

// Weight gradient (stride S = 1 or 2) on two-dimensional output tiles, every tap at
// once: a workgroup owns a chunk of kWgTW output columns by `rows` output
// rows of one image and a block of CB input channels, and walks it TH
// rows at a time.  Each step stages the dz rows and the input rows it needs
// (S * TH + 3 - S rows with the halo) in LDS once, channel-major so that the
// eight consecutive pixels an MFMA operand fragment takes are one 16-byte
// read; the input is stored three times, one copy per horizontal tap kx
// holding the input columns S * x + kx - 1 of output columns x, so that
// every tap reads aligned vectors.  The contraction runs over the
// 32 pixels of one output row per MFMA; M = co (MT tiles of 16), N = the
// 9 * CB (tap, channel) columns of the block, spread over the four waves
// column tile by column tile.  Partials and bias partials have the layout
// of conv_wgrad_kernel (chunk-major rows of 9 * cin), so the same reduction
// follows; the workgroups of channel block 0 sum the bias partials.
constexpr int kWgTW = 32;

template <int MT, int CB, int TH, int S>
__global__ __launch_bounds__(kThreads) void conv_wgrad_tiled_kernel(ConvIn in, int ho, int wo,
                                                                    const uint16_t* __restrict__ dz, int coutp,
                                                                    int rows, int bands,
                                                                    float* __restrict__ partial,
                                                                    float* __restrict__ bpart)
{
    // staged input rows (S * TH + 3 - S for stride S); 8-pixel groups per row;
    // input pixels an item of eight output columns reads
    constexpr int IH = S * TH + 3 - S, Q = kWgTW / 8, NP = 7 * S + 3;
    constexpr int TCT = (9 * CB + 15) / 16, NCT = (TCT + 3) / 4;   // column tiles: all, per wave
    // channel strides padded to an odd number of 16-byte units, so that the
    // 16 channels an operand fetch reads start in different banks
    constexpr int SI = IH * Q + 1, SD = TH * Q + 1;
    __shared__ uint4 s_in[3 * CB * SI];   // [kx][c][iy][q]: input column S * (x0 + 8q + j) + kx - 1, j < 8
    __shared__ uint4 s_dz[MT * 16 * SD];                      // [co][oy][q]
    const int cin = in.ca + in.cb, K = 9 * cin;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, r = lane & 15;
    const int x0 = blockIdx.x * kWgTW, band = blockIdx.y % bands, n = blockIdx.y / bands;
    const int cb0 = blockIdx.z * CB, y_end = min(ho, (band + 1) * rows);
    const bool bias = blockIdx.z == 0;   // uniform per workgroup
    for (int e = tid; e < MT * 16 * SD; e += kThreads)         // channels past coutp stay zero
        if (e >= coutp * SD) s_dz[e] = make_uint4(0, 0, 0, 0);
    // this lane's LDS offset (in 16-byte units, row 0) per column tile
    int boff[NCT];
    bool bval[NCT];
#pragma unroll
    for (int i = 0; i < NCT; ++i) {
        const int ct = wave + 4 * i, kl = 16 * ct + r, tap = kl / CB, c = kl - tap * CB;
        bval[i] = ct < TCT;
        const int ky = tap < 9 ? tap / 3 : 0, kx = tap < 9 ? tap - 3 * (tap / 3) : 0;
        boff[i] = (tap < 9 && cb0 + c < cin) ? (kx * CB + c) * SI + ky * Q + g : -1;
    }
    f4 acc[MT][NCT];
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int i = 0; i < NCT; ++i) acc[t][i] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;
    auto half = [](const uint4& v, int ch) -> uint32_t {
        const uint32_t w = ch < 2 ? v.x : ch < 4 ? v.y : ch < 6 ? v.z : v.w;
        return (ch & 1) ? w >> 16 : w & 0xFFFFu;
    };
    for (int y0 = band * rows; y0 < y_end; y0 += TH) {
        // input rows S * y0 - 1 .. : item (q, iy, channel group), so that
        // neighbouring threads write neighbouring 16-byte units
        for (int e = tid; e < IH * Q * (CB / 8); e += kThreads) {
            const int q = e % Q, iy = (e / Q) % IH, cg = e / (Q * IH);
            const int c8 = cb0 + 8 * cg, y = S * y0 - 1 + iy, xb = S * (x0 + 8 * q) - 1;
            uint4 px[NP];
#pragma unroll
            for (int m = 0; m < NP; ++m)
                px[m] = c8 < cin ? __builtin_bit_cast(uint4, gather8(in, n, y, xb + m, c8)) : make_uint4(0, 0, 0, 0);
#pragma unroll
            for (int kx = 0; kx < 3; ++kx)
#pragma unroll
                for (int ch = 0; ch < 8; ++ch) {
                    uint4 v;
                    v.x = half(px[kx], ch) | half(px[S + kx], ch) << 16;
                    v.y = half(px[2 * S + kx], ch) | half(px[3 * S + kx], ch) << 16;
                    v.z = half(px[4 * S + kx], ch) | half(px[5 * S + kx], ch) << 16;
                    v.w = half(px[6 * S + kx], ch) | half(px[7 * S + kx], ch) << 16;
                    s_in[(kx * CB + 8 * cg + ch) * SI + iy * Q + q] = v;
                }
        }
        // dz rows y0 .. y0 + TH - 1 (zero past the image): item (q, oy, channel group)
        for (int e = tid; e < TH * Q * (coutp / 8); e += kThreads) {
            const int q = e % Q, oy = (e / Q) % TH, cg = e / (Q * TH);
            const int y = y0 + oy, xb = x0 + 8 * q;
            uint4 px[8];
#pragma unroll
            for (int m = 0; m < 8; ++m)
                px[m] = (y < y_end && xb + m < wo)
                            ? *reinterpret_cast<const uint4*>(dz + (((int64_t)n * ho + y) * wo + xb + m) * coutp + 8 * cg)
                            : make_uint4(0, 0, 0, 0);
#pragma unroll
            for (int ch = 0; ch < 8; ++ch) {
                uint4 v;
                v.x = half(px[0], ch) | half(px[1], ch) << 16;
                v.y = half(px[2], ch) | half(px[3], ch) << 16;
                v.z = half(px[4], ch) | half(px[5], ch) << 16;
                v.w = half(px[6], ch) | half(px[7], ch) << 16;
                s_dz[(8 * cg + ch) * SD + oy * Q + q] = v;
            }
        }
        __syncthreads();
        if (bias && tid < coutp) {
#pragma unroll
            for (int e = 0; e < TH * Q; ++e) {
                const uint4 v = s_dz[tid * SD + e];
                bsum += ((bf2f(v.x & 0xFFFFu) + bf2f(v.x >> 16)) + (bf2f(v.y & 0xFFFFu) + bf2f(v.y >> 16))) +
                        ((bf2f(v.z & 0xFFFFu) + bf2f(v.z >> 16)) + (bf2f(v.w & 0xFFFFu) + bf2f(v.w >> 16)));
            }
        }
#pragma unroll
        for (int oy = 0; oy < TH; ++oy) {
            bf16x8 A[MT];
#pragma unroll
            for (int t = 0; t < MT; ++t)
                A[t] = __builtin_bit_cast(bf16x8, s_dz[(t * 16 + r) * SD + oy * Q + g]);
#pragma unroll
            for (int i = 0; i < NCT; ++i) {
                if (!bval[i]) continue;   // uniform per wave
                const bf16x8 B = boff[i] >= 0 ? __builtin_bit_cast(bf16x8, s_in[boff[i] + S * oy * Q]) : zero8();
#pragma unroll
                for (int t = 0; t < MT; ++t) acc[t][i] = mfma(A[t], B, acc[t][i]);
            }
        }
        __syncthreads();
    }
    const int64_t chunk = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    if (bias && tid < coutp) bpart[chunk * coutp + tid] = bsum;
#pragma unroll
    for (int i = 0; i < NCT; ++i) {
        if (!bval[i]) continue;
        const int kl = 16 * (wave + 4 * i) + r, tap = kl / CB, c = kl - tap * CB;
        if (tap >= 9 || cb0 + c >= cin) continue;
        const int k = tap * cin + cb0 + c;
#pragma unroll
        for (int t = 0; t < MT; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j) partial[(chunk * (MT * 16) + t * 16 + 4 * g + j) * K + k] = acc[t][i][j];
    }
}

// grad[co][k] = sum over chunks of partial[chunk][co][k]: a workgroup takes
// 64 consecutive (co, k) entries, wave w adds chunks w, w + 4, ... in order,
// then the four wave sums are added in order (deterministic).  The last
// workgroup does the same for the bias: db[c] = sum over chunks of
// bpart[chunk][c] (c < cout <= 64).
__global__ __launch_bounds__(kThreads) void wgrad_reduce_kernel(const float* __restrict__ partial, int chunks,
                                                                int mpad, int cout, int K, float* __restrict__ grad,
                                                                const float* __restrict__ bpart, int coutp,
                                                                float* __restrict__ db)
{
    __shared__ float s[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (blockIdx.x == gridDim.x - 1) {
        float r = 0.0f;
        if (lane < cout)
#pragma unroll 8
            for (int k = w; k < chunks; k += 4) r += bpart[(int64_t)k * coutp + lane];
        s[w][lane] = r;
        __syncthreads();
        if (threadIdx.x < cout) db[lane] = ((s[0][lane] + s[1][lane]) + s[2][lane]) + s[3][lane];
        return;
    }
    const int i = blockIdx.x * 64 + lane;
    float r = 0.0f;
    if (i < cout * K) {
        const int co = i / K, k = i - co * K;
#pragma unroll 8
        for (int c = w; c < chunks; c += 4) r += partial[((int64_t)c * mpad + co) * K + k];
    }
    s[w][lane] = r;
    __syncthreads();
    if (w == 0 && i < cout * K) grad[i] = ((s[0][lane] + s[1][lane]) + s[2][lane]) + s[3][lane];
}

// ---------------------------------------------------------------- elementwise

// Relative-MSE loss over RGB: per-block partial sums of (o-t)^2/(t^2+0.01)
// and the gradient 2(o-t)/(t^2+0.01)/(3P) written as BF16 with 8 channels.
__global__ __launch_bounds__(kThreads) void loss_kernel(const float* __restrict__ out,
                                                        const float* __restrict__ target, int64_t P,
                                                        uint16_t* __restrict__ dz, float* __restrict__ partial)
{
    __shared__ float s[kThreads];
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    float l = 0.0f;
    if (p < P) {
        const float scale = 2.0f / (3.0f * (float)P);
        uint16_t g8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int c = 0; c < 3; ++c) {
            const float t = target[p * 3 + c], d = out[p * 3 + c] - t;
            const float inv = 1.0f / (t * t + 0.01f);
            l = fmaf(d * d, inv, l);
            g8[c] = f2bf(scale * d * inv);
        }
        uint4 v;
        v.x = g8[0] | ((uint32_t)g8[1] << 16);
        v.y = g8[2];
        v.z = 0;
        v.w = 0;
        *reinterpret_cast<uint4*>(dz + p * 8) = v;
    }
    s[threadIdx.x] = l;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(kThreads) void loss_final_kernel(const float* __restrict__ partial, int nb,
                                                              int64_t P, float* __restrict__ loss)
{
    __shared__ float s[kThreads];
    float a = 0.0f;
    for (int i = threadIdx.x; i < nb; i += kThreads) a += partial[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = s[0] / (3.0f * (float)P);
}

// Adam (Kingma & Ba): FP32 master weights, first and second moments,
// bias corrections c1 = 1 - beta1^t, c2 = 1 - beta2^t; writes the BF16 copy.
__global__ void adam_kernel(float* __restrict__ p, uint16_t* __restrict__ pb, float* __restrict__ m,
                            float* __restrict__ v, const float* __restrict__ grad, uint64_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float x = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = x;
    pb[i] = f2bf(x);
}

__global__ void to_bf16_kernel(const float* __restrict__ p, uint16_t* __restrict__ pb, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) pb[i] = f2bf(p[i]);
}

// Network input from a render: (r, g, b, depth fraction, transmittance, 0, 0, 0).
__global__ void pack_kernel(const float* __restrict__ rgba, const float* __restrict__ aov, uint64_t P,
                            uint16_t* __restrict__ x)
{
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    uint4 v;
    v.x = f2bf(rgba[4 * p]) | ((uint32_t)f2bf(rgba[4 * p + 1]) << 16);
    v.y = f2bf(rgba[4 * p + 2]) | ((uint32_t)f2bf(aov[2 * p]) << 16);
    v.z = f2bf(aov[2 * p + 1]);
    v.w = 0;
    *reinterpret_cast<uint4*>(x + 8 * p) = v;
}

// ---------------------------------------------------------------- host side

inline unsigned blocks(uint64_t n, unsigned t = kThreads) { return (unsigned)((n + t - 1) / t); }

vdbc_status check(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VDBC_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
    return VDBC_OK;
}

bool aligned16(const void* p) { return p == nullptr || (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Dynamic LDS past 64 KiB needs the kernel's limit raised first; false
// (and the error cleared) where the device refuses, so that the caller can
// take a variant that needs less.
bool allow_lds(const void* kernel, size_t bytes)
{
    if (bytes <= 65536) return true;
    if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess) return true;
    (void)hipGetLastError();
    return false;
}

vdbc_status conv_fwd(const ConvIn& in, int stride, const uint16_t* w, const float* bias, int cout,
                     int relu, uint16_t* out_bf, float* out_f, const uint16_t* resid, hipStream_t st)
{
    const int hv = in.up ? 2 * in.hs : in.hs, wv = in.up ? 2 * in.ws : in.ws;
    const int ho = (hv - 1) / stride + 1, wo = (wv - 1) / stride + 1;
    const uint64_t P = (uint64_t)in.n * ho * wo;
    const unsigned tiles_y = (unsigned)((ho + kFwdTH - 1) / kFwdTH);
    if (stride == 1 && tiles_y <= 65535u && in.n <= 65535) {   // grid y and z limits
        const dim3 grid((wo + kFwdTW - 1) / kFwdTW, tiles_y, in.n);
        const int nt = cout <= 16 ? 1 : cout <= 32 ? 2 : 4;
        const size_t win = (size_t)(kFwdTH + 2) * (kFwdTW + 2) * ((in.ca + in.cb) / 8 + 1) * 16;
        const size_t epi = (size_t)(nt < 2 ? nt : 2) * 16 * kEpiStride * 4;
        // the staged epilogue for BF16 output in groups of four channels
        const bool staged = out_bf && !out_f && cout % 4 == 0 && (reinterpret_cast<uintptr_t>(out_bf) & 7u) == 0;
        const size_t lds = staged && epi > win ? epi : win;
#define VDBC_FWD_TILED(NTV, S)                                                                                    \
    hipLaunchKernelGGL((conv_fwd_tiled_kernel<NTV, S>), grid, dim3(kThreads), lds, st, in, w, bias, cout, ho, wo, \
                       relu, out_bf, out_f, resid)
        if (staged) {
            if (nt == 1)
                VDBC_FWD_TILED(1, true);
            else if (nt == 2)
                VDBC_FWD_TILED(2, true);
            else
                VDBC_FWD_TILED(4, true);
        } else {
            if (nt == 1)
                VDBC_FWD_TILED(1, false);
            else if (nt == 2)
                VDBC_FWD_TILED(2, false);
            else
                VDBC_FWD_TILED(4, false);
        }
#undef VDBC_FWD_TILED
        return check("conv3x3 forward");
    }
    const unsigned gb = blocks(P, 64 * kConvTiles);
    if (cout <= 16)   // one channel tile: one pixel tile per wave keeps more workgroups in flight
        hipLaunchKernelGGL((conv_fwd_kernel<1, 1>), dim3(blocks(P, 64)), dim3(kThreads), 0, st, in, w, bias, cout,
                           stride, ho, wo, relu, out_bf, out_f, resid);
    else if (cout <= 32)
        hipLaunchKernelGGL((conv_fwd_kernel<2, kConvTiles>), dim3(gb), dim3(kThreads), 0, st, in, w, bias, cout,
                           stride, ho, wo, relu, out_bf, out_f, resid);
    else
        hipLaunchKernelGGL((conv_fwd_kernel<4, kConvTiles>), dim3(gb), dim3(kThreads), 0, st, in, w, bias, cout,
                           stride, ho, wo, relu, out_bf, out_f, resid);
    return check("conv3x3 forward");
}

// 2 x 2 sums through the ReLU backward into BF16 dz at half resolution.
DgradOut pool_out(uint16_t* dz, int dz_stride, const uint16_t* y, int y_stride)
{
    return DgradOut{nullptr, 0, 0, 0, dz, dz_stride, y, y_stride, nullptr, 0, 1};
}
// Every channel as FP32 (stride `cin`).
DgradOut fp32_out(float* dx, int cin) { return DgradOut{dx, cin, 0, cin, nullptr, 0, nullptr, 0, nullptr, 0}; }
// Channels [split, cin) through the ReLU backward into BF16 dz (see DgradOut).
DgradOut relu_out(float* dx, int split, uint16_t* dz, int dz_stride, const uint16_t* y, int y_stride,
                  const float* add = nullptr, int add_stride = 0)
{
    return DgradOut{dx, split, 0, split, dz, dz_stride, y, y_stride, add, add_stride};
}

vdbc_status conv_dgrad(const uint16_t* dz, int coutp, int cout, int n, int ho, int wo, const uint16_t* w,
                       int cin, int stride, int hv, int wv, const DgradOut& out_in, uint16_t* wt,
                       hipStream_t st, bool wt_ready = false)
{
    if (out_in.split % 4) return fail(VDBC_E_INVALID, "data gradient: split must be a multiple of 4");
    DgradOut out = out_in;
    auto al8 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; };
    const bool fp_ok = out.split == 0 || (aligned16(out.dx) && out.dx_stride % 4 == 0);
    const bool bf_ok = out.split >= cin || ((!out.add || (aligned16(out.add) && out.add_stride % 4 == 0)) &&
                                            al8(out.y) && al8(out.dz) && out.y_stride % 4 == 0 &&
                                            out.dz_stride % 4 == 0);
    out.vec = fp_ok && bf_ok;
    if (!wt_ready)
        hipLaunchKernelGGL(transpose_weights_kernel, dim3(blocks((uint64_t)cin * 9 * coutp)), dim3(kThreads), 0, st,
                           w, cin, cout, coutp, wt);
    const uint64_t Q = (uint64_t)n * hv * wv;
    const unsigned gb = blocks(Q, 64 * kConvTiles);
    const unsigned tiles_y = (unsigned)((hv + kFwdTH - 1) / kFwdTH);
    const bool tiled = stride == 1 && hv == ho && wv == wo && tiles_y <= 65535u && n <= 65535;   // grid y, z limits
    if (out.pool && !(tiled && hv % 2 == 0 && wv % 2 == 0 && out.split == 0))
        return fail(VDBC_E_INVALID, "pooled data gradient needs stride 1, even sizes and the tiled kernel");
    if (tiled) {
        const dim3 grid((wv + kFwdTW - 1) / kFwdTW, tiles_y, n);
        const int nt = cin <= 16 ? 1 : cin <= 32 ? 2 : 4;
        const size_t win = (size_t)(kFwdTH + 2) * (kFwdTW + 2) * (coutp / 8 + 1) * 16;
        const size_t epi = (size_t)(nt < 2 ? nt : 2) * 16 * kEpiStride * 4;   // two channel tiles per pass
        const size_t lds = win > epi ? win : epi;
        // the staged epilogue where the LDS allows it (the pooled one stays direct)
        const void* kern = nt == 1   ? reinterpret_cast<const void*>(&conv_dgrad_tiled_kernel<1, true>)
                           : nt == 2 ? reinterpret_cast<const void*>(&conv_dgrad_tiled_kernel<2, true>)
                                     : reinterpret_cast<const void*>(&conv_dgrad_tiled_kernel<4, true>);
        const bool staged = !out.pool && allow_lds(kern, lds);
#define VDBC_DGRAD_TILED(NTV, S, L)                                                                              \
    hipLaunchKernelGGL((conv_dgrad_tiled_kernel<NTV, S>), grid, dim3(kThreads), L, st, dz, coutp, ho, wo, wt, cin, \
                       out)
        if (staged) {
            if (nt == 1)
                VDBC_DGRAD_TILED(1, true, lds);
            else if (nt == 2)
                VDBC_DGRAD_TILED(2, true, lds);
            else
                VDBC_DGRAD_TILED(4, true, lds);
        } else {
            if (nt == 1)
                VDBC_DGRAD_TILED(1, false, win);
            else if (nt == 2)
                VDBC_DGRAD_TILED(2, false, win);
            else
                VDBC_DGRAD_TILED(4, false, win);
        }
#undef VDBC_DGRAD_TILED
        return check("conv3x3 data gradient");
    }
    if (stride == 2 && tiles_y <= 65535u && n <= 65535) {
        const dim3 grid((wv + kFwdTW - 1) / kFwdTW, tiles_y, n);
        size_t lds = (size_t)(kFwdTH / 2 + 1) * (kFwdTW / 2 + 1) * (coutp / 8 + 1) * 16;
        if (cin <= 32) {   // the staged epilogue of one or two channel tiles
            const size_t epi = (size_t)(cin <= 16 ? 16 : 32) * kEpiStride * 4;
            lds = lds > epi ? lds : epi;
        }
        if (cin <= 16)
            hipLaunchKernelGGL((conv_dgrad_s2_kernel<1>), grid, dim3(kThreads), lds, st, dz, coutp, ho, wo, wt, cin,
                               hv, wv, out);
        else if (cin <= 32)
            hipLaunchKernelGGL((conv_dgrad_s2_kernel<2>), grid, dim3(kThreads), lds, st, dz, coutp, ho, wo, wt, cin,
                               hv, wv, out);
        else
            hipLaunchKernelGGL((conv_dgrad_s2_kernel<4>), grid, dim3(kThreads), lds, st, dz, coutp, ho, wo, wt, cin,
                               hv, wv, out);
        return check("conv3x3 data gradient");
    }
    if (cin <= 16)
        hipLaunchKernelGGL((conv_dgrad_kernel<1, kConvTiles>), dim3(gb), dim3(kThreads), 0, st, dz, coutp, n, ho,
                           wo, wt, cin, stride, hv, wv, out);
    else if (cin <= 32)
        hipLaunchKernelGGL((conv_dgrad_kernel<2, kConvTiles>), dim3(gb), dim3(kThreads), 0, st, dz, coutp, n, ho,
                           wo, wt, cin, stride, hv, wv, out);
    else   // four channel tiles: two pixel tiles per wave (fewer registers, more waves in flight)
        hipLaunchKernelGGL((conv_dgrad_kernel<4, 2>), dim3(blocks(Q, 128)), dim3(kThreads), 0, st, dz, coutp, n, ho,
                           wo, wt, cin, stride, hv, wv, out);
    return check("conv3x3 data gradient");
}

// 16-channel output tiles of the weight-gradient kernel launched for `cout`
// output channels: 1, 2 or 4 (33..64 channels take the four-tile kernel, so
// its partial rows are 64 apart).
int wgrad_mt(int cout) { return cout <= 16 ? 1 : cout <= 32 ? 2 : 4; }

// Launch plan of the tiled weight-gradient kernel: channel block
// CB (8, 16 or 32; blocks of 64 channels with two rows per step measured
// 1 % slower), TH rows per step, and output rows per chunk halved from 64
// (down to TH) while the launch would have fewer than kWgTiledGroups
// workgroups (targets of 256 or 1024 were 5-7 % slower per training step:
// fewer workgroups fill the chip less, more write more partials); stride 2
// takes two output rows per step.  `ok` is false for launches past the grid's
// y and z limits; those take conv_wgrad_kernel.
constexpr uint64_t kWgTiledGroups = 512;

struct WgradTiled {
    int cb, th, rows, bands, cols, cblocks;
    uint64_t chunks;
    bool ok;
};

WgradTiled wgrad_tiled_plan(const ConvIn& in, int stride, int cout)
{
    WgradTiled p{};
    const int cin = in.ca + in.cb;
    const int hv = in.up ? 2 * in.hs : in.hs, wv = in.up ? 2 * in.ws : in.ws;
    const int ho = (hv - 1) / stride + 1, wo = (wv - 1) / stride + 1;
    p.cb = cin <= 8 ? 8 : cin <= 16 ? 16 : 32;
    p.th = stride == 1 ? 4 : 2;
    p.cols = (wo + kWgTW - 1) / kWgTW;
    p.cblocks = (cin + p.cb - 1) / p.cb;
    auto groups = [&](int rows) { return (uint64_t)in.n * ((ho + rows - 1) / rows) * p.cols * p.cblocks; };
    p.rows = 64;
    while (p.rows > p.th && groups(p.rows) < kWgTiledGroups) p.rows /= 2;
    p.bands = (ho + p.rows - 1) / p.rows;
    p.chunks = (uint64_t)in.n * p.bands * p.cols;
    p.ok = (stride == 1 || stride == 2) && (uint64_t)in.n * p.bands <= 65535u && p.cblocks <= 65535;
    return p;
}

// Weight-gradient chunks of a launch: the tiled kernel's or conv_wgrad_kernel's.
uint64_t wgrad_chunks(const ConvIn& in, int stride, int cout)
{
    const WgradTiled tp = wgrad_tiled_plan(in, stride, cout);
    if (tp.ok) return tp.chunks;
    const int hv = in.up ? 2 * in.hs : in.hs, wv = in.up ? 2 * in.ws : in.ws;
    const uint64_t P = (uint64_t)in.n * ((hv - 1) / stride + 1) * ((wv - 1) / stride + 1);
    const uint64_t c = wgrad_chunk(P, 9 * (in.ca + in.cb));
    return (P + c - 1) / c;
}

// Floats of the weight-gradient partials followed by the bias partials
// (chunks x coutp, coutp <= 64).
uint64_t wgrad_partial_floats(const ConvIn& in, int stride, int cout)
{
    const uint64_t chunks = wgrad_chunks(in, stride, cout);
    const int mpad = wgrad_mt(cout) * 16;
    return chunks * mpad * 9ull * (in.ca + in.cb) + chunks * 64ull;
}

template <int MT, int CB>
void launch_wgrad_tiled(const WgradTiled& p, const ConvIn& in, int ho, int wo, const uint16_t* dz, int coutp,
                        float* partial, float* bpart, hipStream_t st)
{
    const dim3 grid(p.cols, in.n * p.bands, p.cblocks);
    if (p.th == 4)   // stride 1
        hipLaunchKernelGGL((conv_wgrad_tiled_kernel<MT, CB, 4, 1>), grid, dim3(kThreads), 0, st, in, ho, wo, dz,
                           coutp, p.rows, p.bands, partial, bpart);
    else             // stride 2, two output rows per step
        hipLaunchKernelGGL((conv_wgrad_tiled_kernel<MT, CB, 2, 2>), grid, dim3(kThreads), 0, st, in, ho, wo, dz,
                           coutp, p.rows, p.bands, partial, bpart);
}

template <int MT>
void launch_wgrad_tiled_mt(const WgradTiled& p, const ConvIn& in, int ho, int wo, const uint16_t* dz, int coutp,
                           float* partial, float* bpart, hipStream_t st)
{
    if (p.cb == 8)
        launch_wgrad_tiled<MT, 8>(p, in, ho, wo, dz, coutp, partial, bpart, st);
    else if (p.cb == 16)
        launch_wgrad_tiled<MT, 16>(p, in, ho, wo, dz, coutp, partial, bpart, st);
    else
        launch_wgrad_tiled<MT, 32>(p, in, ho, wo, dz, coutp, partial, bpart, st);
}

vdbc_status conv_wgrad(const ConvIn& in, int stride, const uint16_t* dz, int coutp, int cout, float* dw,
                       float* db, float* partial, uint64_t partial_floats, hipStream_t st)
{
    const uint64_t need = wgrad_partial_floats(in, stride, cout);
    if (need > partial_floats)
        return fail(VDBC_E_BUFFER_TOO_SMALL, "weight-gradient partials need %llu floats, the workspace holds %llu",
                    (unsigned long long)need, (unsigned long long)partial_floats);
    const int cin = in.ca + in.cb, K = 9 * cin;
    const int hv = in.up ? 2 * in.hs : in.hs, wv = in.up ? 2 * in.ws : in.ws;
    const int ho = (hv - 1) / stride + 1, wo = (wv - 1) / stride + 1;
    const int64_t P = (int64_t)in.n * ho * wo;
    const int chunk = wgrad_chunk(P, K);
    const int mt = wgrad_mt(cout);
    const WgradTiled tp = wgrad_tiled_plan(in, stride, cout);
    const unsigned chunks = (unsigned)wgrad_chunks(in, stride, cout);
    dim3 grid(chunks, (K + 63) / 64);
    float* bpart = partial + (uint64_t)chunks * (mt * 16) * K;
    if (tp.ok) {
        if (mt == 1)
            launch_wgrad_tiled_mt<1>(tp, in, ho, wo, dz, coutp, partial, bpart, st);
        else if (mt == 2)
            launch_wgrad_tiled_mt<2>(tp, in, ho, wo, dz, coutp, partial, bpart, st);
        else
            launch_wgrad_tiled_mt<4>(tp, in, ho, wo, dz, coutp, partial, bpart, st);
    } else if (mt == 1)
        hipLaunchKernelGGL(conv_wgrad_kernel<1>, grid, dim3(kThreads), 0, st, in, stride, ho, wo, dz, coutp, chunk, partial,
                           bpart);
    else if (mt == 2)
        hipLaunchKernelGGL(conv_wgrad_kernel<2>, grid, dim3(kThreads), 0, st, in, stride, ho, wo, dz, coutp, chunk, partial,
                           bpart);
    else   // mt == 4
        hipLaunchKernelGGL(conv_wgrad_kernel<4>, grid, dim3(kThreads), 0, st, in, stride, ho, wo, dz, coutp, chunk, partial,
                           bpart);
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((unsigned)(((uint64_t)cout * K + 63) / 64) + 1), dim3(kThreads), 0, st,
                       partial, (int)chunks, mt * 16, cout, K, dw, bpart, coutp, db);
    return check("conv3x3 weight gradient");
}

// Workspace carving for the whole network at n x h x w.
struct NetLayout {
    uint64_t c1, c2, c3, c4, c5, out, dz6, dz5, dcat, dz4, dz3, dz2, dz1, wt, partial,
        lpart, grad, total;
};

uint64_t al(uint64_t x) { return (x + 255u) & ~uint64_t(255u); }

// The largest weight-gradient partials of the network's six layers, with the
// inputs, strides and output channels of the training step's backward pass.
uint64_t net_partial_floats(uint32_t n, uint32_t h, uint32_t w)
{
    const int N = (int)n, H = (int)h, W = (int)w;
    const uint64_t f[6] = {
        wgrad_partial_floats(ConvIn{nullptr, nullptr, 32, 0, 0, N, H, W}, 1, 3),
        wgrad_partial_floats(ConvIn{nullptr, nullptr, 32, 32, 0, N, H, W}, 1, 32),
        wgrad_partial_floats(ConvIn{nullptr, nullptr, 64, 0, 1, N, H / 2, W / 2}, 1, 32),
        wgrad_partial_floats(ConvIn{nullptr, nullptr, 64, 0, 0, N, H / 2, W / 2}, 1, 64),
        wgrad_partial_floats(ConvIn{nullptr, nullptr, 32, 0, 0, N, H, W}, 2, 64),
        wgrad_partial_floats(ConvIn{nullptr, nullptr, 8, 0, 0, N, H, W}, 1, 32)};
    uint64_t m = 0;
    for (uint64_t x : f) m = x > m ? x : m;
    return m;
}

NetLayout net_layout(uint32_t n, uint32_t h, uint32_t w, bool training)
{
    const uint64_t P = (uint64_t)n * h * w, Ph = P / 4;
    NetLayout L{};
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t at = o;
        o += al(bytes);
        return at;
    };
    L.c1 = take(P * 32 * 2);
    L.c2 = take(Ph * 64 * 2);
    L.c3 = take(Ph * 64 * 2);
    L.c4 = take(P * 32 * 2);
    L.c5 = take(P * 32 * 2);
    if (training) {
        L.out = take(P * 3 * 4);
        L.dz6 = take(P * 8 * 2);
        L.dz5 = take(P * 32 * 2);
        L.dcat = take(P * 32 * 4);   // the c1 half of the concat's gradient
        L.dz4 = take(P * 32 * 2);
        L.dz3 = take(Ph * 64 * 2);
        L.dz2 = take(Ph * 64 * 2);
        L.dz1 = take(P * 32 * 2);
        L.wt = take(5 * 64 * 9 * 64 * 2);   // transposed weights of the five data gradients
        L.partial = take(net_partial_floats(n, h, w) * 4);
        L.lpart = take((P + kThreads - 1) / kThreads * 4 + 16);
        L.grad = take(nn::param_count() * 4);
    }
    L.total = o;
    return L;
}

vdbc_status check_net_args(uint32_t n, uint32_t h, uint32_t w)
{
    if (n == 0 || h == 0 || w == 0 || (h & 1u) || (w & 1u))
        return fail(VDBC_E_INVALID, "denoiser needs n >= 1 and even h, w >= 2");
    if ((uint64_t)n * h * w > (1ull << 31)) return fail(VDBC_E_INVALID, "too many pixels");
    return VDBC_OK;
}

// Forward pass into the workspace; `out` gets the FP32 RGB result.
vdbc_status net_forward(const float* params, const uint16_t* wb, const uint16_t* x, uint32_t n, uint32_t h,
                        uint32_t w, float* out, uint8_t* ws, const NetLayout& L, hipStream_t st)
{
    using namespace nn;
    auto Wl = [&](int l) { return wb + weight_offset(l); };
    auto Bl = [&](int l) { return params + bias_offset(l); };
    uint16_t* c1 = reinterpret_cast<uint16_t*>(ws + L.c1);
    uint16_t* c2 = reinterpret_cast<uint16_t*>(ws + L.c2);
    uint16_t* c3 = reinterpret_cast<uint16_t*>(ws + L.c3);
    uint16_t* c4 = reinterpret_cast<uint16_t*>(ws + L.c4);
    uint16_t* c5 = reinterpret_cast<uint16_t*>(ws + L.c5);
    const int H = (int)h, W = (int)w, N = (int)n;
    vdbc_status s;
    if ((s = conv_fwd(ConvIn{x, nullptr, 8, 0, 0, N, H, W}, 1, Wl(0), Bl(0), 32, 1, c1, nullptr, nullptr, st)))
        return s;
    if ((s = conv_fwd(ConvIn{c1, nullptr, 32, 0, 0, N, H, W}, 2, Wl(1), Bl(1), 64, 1, c2, nullptr, nullptr, st)))
        return s;
    if ((s = conv_fwd(ConvIn{c2, nullptr, 64, 0, 0, N, H / 2, W / 2}, 1, Wl(2), Bl(2), 64, 1, c3, nullptr,
                      nullptr, st)))
        return s;
    if ((s = conv_fwd(ConvIn{c3, nullptr, 64, 0, 1, N, H / 2, W / 2}, 1, Wl(3), Bl(3), 32, 1, c4, nullptr,
                      nullptr, st)))
        return s;
    if ((s = conv_fwd(ConvIn{c1, c4, 32, 32, 0, N, H, W}, 1, Wl(4), Bl(4), 32, 1, c5, nullptr, nullptr, st)))
        return s;
    return conv_fwd(ConvIn{c5, nullptr, 32, 0, 0, N, H, W}, 1, Wl(5), Bl(5), 3, 0, nullptr, out, x, st);
}

}  // namespace
}  // namespace vdbc

using namespace vdbc;

extern "C" vdbc_status vdbc_nn_param_count(uint64_t* count)
{
    clear_error();
    if (!count) return fail(VDBC_E_INVALID, "null argument");
    *count = nn::param_count();
    return VDBC_OK;
}

extern "C" vdbc_status vdbc_nn_to_bf16(const float* params, uint16_t* wbf16, void* stream)
{
    clear_error();
    if (!params || !wbf16) return fail(VDBC_E_INVALID, "null argument");
    const uint64_t n = nn::param_count();
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks(n)), dim3(kThreads), 0, static_cast<hipStream_t>(stream),
                       params, wbf16, n);
    return check("vdbc_nn_to_bf16");
}

extern "C" vdbc_status vdbc_denoise_workspace(uint32_t n, uint32_t h, uint32_t w, uint32_t training,
                                              uint64_t* bytes)
{
    clear_error();
    if (!bytes) return fail(VDBC_E_INVALID, "null argument");
    vdbc_status s = check_net_args(n, h, w);
    if (s) return s;
    *bytes = net_layout(n, h, w, training != 0).total;
    return VDBC_OK;
}

extern "C" vdbc_status vdbc_denoise_pack(const float* rgba, const float* aov, uint64_t pixels, uint16_t* x,
                                         void* stream)
{
    clear_error();
    if (pixels && (!rgba || !aov || !x)) return fail(VDBC_E_INVALID, "null argument");
    if (!aligned16(x)) return fail(VDBC_E_INVALID, "x must be 16-byte aligned");
    if (pixels == 0) return VDBC_OK;
    hipLaunchKernelGGL(pack_kernel, dim3(blocks(pixels)), dim3(kThreads), 0, static_cast<hipStream_t>(stream),
                       rgba, aov, pixels, x);
    return check("vdbc_denoise_pack");
}

extern "C" vdbc_status vdbc_denoise(const float* params, const uint16_t* wbf16, const uint16_t* x, uint32_t n,
                                    uint32_t h, uint32_t w, float* out, void* ws, uint64_t ws_bytes, void* stream)
{
    clear_error();
    vdbc_status s = check_net_args(n, h, w);
    if (s) return s;
    if (!params || !wbf16 || !x || !out || !ws) return fail(VDBC_E_INVALID, "null argument");
    if (!aligned16(wbf16) || !aligned16(x) || (reinterpret_cast<uintptr_t>(ws) & 255u))
        return fail(VDBC_E_INVALID, "wbf16 and x must be 16-byte aligned, ws 256-byte aligned");
    const NetLayout L = net_layout(n, h, w, false);
    if (ws_bytes < L.total)
        return fail(VDBC_E_BUFFER_TOO_SMALL, "denoise workspace needs %llu bytes", (unsigned long long)L.total);
    return net_forward(params, wbf16, x, n, h, w, out, static_cast<uint8_t*>(ws), L,
                       static_cast<hipStream_t>(stream));
}

extern "C" vdbc_status vdbc_denoise_train_step(float* params, uint16_t* wbf16, float* adam_m, float* adam_v,
                                               uint32_t step, float lr, const uint16_t* x, const float* target,
                                               uint32_t n, uint32_t h, uint32_t w, float* loss, float* grad_out,
                                               void* ws, uint64_t ws_bytes, void* stream)
{
    using namespace nn;
    clear_error();
    vdbc_status s = check_net_args(n, h, w);
    if (s) return s;
    if (!params || !wbf16 || !x || !target || !loss || !ws) return fail(VDBC_E_INVALID, "null argument");
    if (step == 0 || !(lr >= 0.0f) || !std::isfinite(lr)) return fail(VDBC_E_INVALID, "step >= 1, finite lr >= 0");
    if (lr > 0.0f && (!adam_m || !adam_v)) return fail(VDBC_E_INVALID, "null Adam state");
    if (!aligned16(wbf16) || !aligned16(x) || (reinterpret_cast<uintptr_t>(ws) & 255u))
        return fail(VDBC_E_INVALID, "wbf16 and x must be 16-byte aligned, ws 256-byte aligned");
    const NetLayout L = net_layout(n, h, w, true);
    if (ws_bytes < L.total)
        return fail(VDBC_E_BUFFER_TOO_SMALL, "training workspace needs %llu bytes", (unsigned long long)L.total);
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint8_t* b = static_cast<uint8_t*>(ws);
    auto U = [&](uint64_t off) { return reinterpret_cast<uint16_t*>(b + off); };
    auto F = [&](uint64_t off) { return reinterpret_cast<float*>(b + off); };
    const int H = (int)h, W = (int)w, N = (int)n;
    const int64_t P = (int64_t)n * h * w;
    float* out = F(L.out);
    float* grad = grad_out ? grad_out : F(L.grad);
    if ((s = net_forward(params, wbf16, x, n, h, w, out, b, L, st))) return s;
    // loss and dL/dout
    const unsigned nb = blocks((uint64_t)P);
    hipLaunchKernelGGL(loss_kernel, dim3(nb), dim3(kThreads), 0, st, out, target, P, U(L.dz6), F(L.lpart));
    hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(kThreads), 0, st, F(L.lpart), (int)nb, P, loss);
    if ((s = check("loss"))) return s;
    auto Wl = [&](int l) { return wbf16 + weight_offset(l); };
    auto gW = [&](int l) { return grad + weight_offset(l); };
    auto gB = [&](int l) { return grad + bias_offset(l); };
    uint16_t *c1 = U(L.c1), *c2 = U(L.c2), *c3 = U(L.c3), *c4 = U(L.c4), *c5 = U(L.c5);
    float* part = F(L.partial);
    const uint64_t pf = net_partial_floats(N, H, W);
    // the five layers' transposed weights in one launch
    uint16_t* wt = U(L.wt);
    auto WT = [&](int l) { return wt + (size_t)l * 64 * 9 * 64; };
    {
        WtJobs j{};
        const int lay[5] = {5, 4, 3, 2, 1}, cin_[5] = {32, 64, 64, 64, 32}, cout_[5] = {3, 32, 32, 64, 64},
                  coutp_[5] = {8, 32, 32, 64, 64};
        for (int i = 0; i < 5; ++i) {
            j.w[i] = Wl(lay[i]);
            j.wt[i] = WT(i);
            j.cin[i] = cin_[i];
            j.cout[i] = cout_[i];
            j.coutp[i] = coutp_[i];
        }
        hipLaunchKernelGGL(transpose_weights_many_kernel, dim3(blocks(64 * 9 * 64), 5), dim3(kThreads), 0, st, j);
        if ((s = check("weight transposes"))) return s;
    }
    // c6: 32 -> 3 (dz6 padded to 8 channels)
    if ((s = conv_wgrad(ConvIn{c5, nullptr, 32, 0, 0, N, H, W}, 1, U(L.dz6), 8, 3, gW(5), gB(5), part, pf, st))) return s;
    if ((s = conv_dgrad(U(L.dz6), 8, 3, N, H, W, Wl(5), 32, 1, H, W, relu_out(nullptr, 0, U(L.dz5), 32, c5, 32),
                        WT(0), st, true)))
        return s;
    // c5: concat(c1, c4) 64 -> 32
    if ((s = conv_wgrad(ConvIn{c1, c4, 32, 32, 0, N, H, W}, 1, U(L.dz5), 32, 32, gW(4), gB(4), part, pf, st))) return s;
    // channels 0..31 of the concat belong to c1 (FP32, added to c2's data
    // gradient below), channels 32..63 to c4 (ReLU backward into dz4)
    if ((s = conv_dgrad(U(L.dz5), 32, 32, N, H, W, Wl(4), 64, 1, H, W, relu_out(F(L.dcat), 32, U(L.dz4), 32, c4, 32),
                        WT(1), st, true)))
        return s;
    // c4: up2(c3) 64 -> 32
    if ((s = conv_wgrad(ConvIn{c3, nullptr, 64, 0, 1, N, H / 2, W / 2}, 1, U(L.dz4), 32, 32, gW(3), gB(3), part, pf,
                        st)))
        return s;
    // the upsample's backward (2 x 2 sums) and c3's ReLU backward in the epilogue
    if ((s = conv_dgrad(U(L.dz4), 32, 32, N, H, W, Wl(3), 64, 1, H, W, pool_out(U(L.dz3), 64, c3, 64), WT(2), st,
                        true)))
        return s;
    // c3: 64 -> 64 at half resolution
    if ((s = conv_wgrad(ConvIn{c2, nullptr, 64, 0, 0, N, H / 2, W / 2}, 1, U(L.dz3), 64, 64, gW(2), gB(2), part, pf,
                        st)))
        return s;
    if ((s = conv_dgrad(U(L.dz3), 64, 64, N, H / 2, W / 2, Wl(2), 64, 1, H / 2, W / 2,
                        relu_out(nullptr, 0, U(L.dz2), 64, c2, 64), WT(3), st, true)))
        return s;
    // c2: 32 -> 64, stride 2
    if ((s = conv_wgrad(ConvIn{c1, nullptr, 32, 0, 0, N, H, W}, 2, U(L.dz2), 64, 64, gW(1), gB(1), part, pf, st)))
        return s;
    if ((s = conv_dgrad(U(L.dz2), 64, 64, N, H / 2, W / 2, Wl(1), 32, 2, H, W,
                        relu_out(nullptr, 0, U(L.dz1), 32, c1, 32, F(L.dcat), 32), WT(4), st, true)))
        return s;
    // c1: 8 -> 32 (no data gradient needed)
    if ((s = conv_wgrad(ConvIn{x, nullptr, 8, 0, 0, N, H, W}, 1, U(L.dz1), 32, 32, gW(0), gB(0), part, pf, st)))
        return s;
    if (lr > 0.0f) {
        const double c1d = 1.0 - std::pow(0.9, (double)step), c2d = 1.0 - std::pow(0.999, (double)step);
        const uint64_t np = param_count();
        hipLaunchKernelGGL(adam_kernel, dim3(blocks(np)), dim3(kThreads), 0, st, params, wbf16, adam_m, adam_v,
                           grad, np, lr, 0.9f, 0.999f, 1e-8f, (float)c1d, (float)c2d);
        if ((s = check("adam"))) return s;
    }
    return VDBC_OK;
}

// ---- single-layer building blocks (parity tests) ----

extern "C" vdbc_status vdbc_conv3x3(const uint16_t* a, uint32_t ca, const uint16_t* b, uint32_t cb,
                                    uint32_t upsample, uint32_t n, uint32_t hs, uint32_t ws_, uint32_t stride,
                                    const uint16_t* w, const float* bias, uint32_t cout, uint32_t relu,
                                    uint16_t* out_bf16, float* out_f32, void* stream)
{
    clear_error();
    if (!a || !w || !bias || (!out_bf16 && !out_f32) || (cb && !b)) return fail(VDBC_E_INVALID, "null argument");
    if (ca % 8 || cb % 8 || ca + cb == 0 || ca + cb > 64 || cout == 0 || cout > 64 || (stride != 1 && stride != 2) ||
        n == 0 || hs == 0 || ws_ == 0)
        return fail(VDBC_E_INVALID, "channels must be multiples of 8 up to 64, cout 1..64, stride 1 or 2");
    if (!aligned16(a) || !aligned16(b) || !aligned16(w)) return fail(VDBC_E_INVALID, "operands must be 16-byte aligned");
    return conv_fwd(ConvIn{a, b, (int)ca, (int)cb, (int)(upsample != 0), (int)n, (int)hs, (int)ws_}, (int)stride, w,
                    bias, (int)cout, (int)relu, out_bf16, out_f32, nullptr, static_cast<hipStream_t>(stream));
}

extern "C" vdbc_status vdbc_conv3x3_grad_workspace(uint32_t cin, uint32_t cout, uint32_t n, uint32_t ho,
                                                   uint32_t wo, uint64_t* bytes)
{
    clear_error();
    if (!bytes || cin == 0 || cin > 64 || cout == 0 || cout > 64) return fail(VDBC_E_INVALID, "bad argument");
    const uint64_t P = (uint64_t)n * ho * wo;
    const uint64_t c = wgrad_chunk(P, 9 * (int)cin), chunks = (P + c - 1) / c;
    // the tiled kernel's chunks for the same output (any cout, stride 1 or 2)
    uint64_t tiled = 0;
    for (int mt_cout : {16, 32, 64}) {
        const WgradTiled t1 = wgrad_tiled_plan(ConvIn{nullptr, nullptr, (int)cin, 0, 0, (int)n, (int)ho, (int)wo},
                                               1, mt_cout);
        const WgradTiled t2 = wgrad_tiled_plan(
            ConvIn{nullptr, nullptr, (int)cin, 0, 0, (int)n, 2 * (int)ho, 2 * (int)wo}, 2, mt_cout);
        tiled = t1.chunks > tiled ? t1.chunks : tiled;
        tiled = t2.chunks > tiled ? t2.chunks : tiled;
    }
    *bytes = al(64ull * 9 * 64 * 2) + al((chunks > tiled ? chunks : tiled) * (64ull * 9 * cin + 64) * 4);
    return VDBC_OK;
}

extern "C" vdbc_status vdbc_conv3x3_dgrad(const uint16_t* dz, uint32_t coutp, uint32_t cout, uint32_t n,
                                          uint32_t ho, uint32_t wo, const uint16_t* w, uint32_t cin,
                                          uint32_t stride, uint32_t hv, uint32_t wv, float* dx, void* ws,
                                          uint64_t ws_bytes, void* stream)
{
    clear_error();
    if (!dz || !w || !dx || !ws) return fail(VDBC_E_INVALID, "null argument");
    if (coutp % 8 || coutp < cout || coutp > 64 || cin % 8 || cin == 0 || cin > 64 || (stride != 1 && stride != 2))
        return fail(VDBC_E_INVALID, "bad channel counts or stride");
    if ((hv - 1) / stride + 1 != ho || (wv - 1) / stride + 1 != wo) return fail(VDBC_E_INVALID, "shape mismatch");
    if (ws_bytes < 64ull * 9 * 64 * 2) return fail(VDBC_E_BUFFER_TOO_SMALL, "workspace too small");
    if (!aligned16(dz) || !aligned16(w) || !aligned16(ws)) return fail(VDBC_E_INVALID, "operands must be 16-byte aligned");
    return conv_dgrad(dz, (int)coutp, (int)cout, (int)n, (int)ho, (int)wo, w, (int)cin, (int)stride, (int)hv,
                      (int)wv, fp32_out(dx, (int)cin), static_cast<uint16_t*>(ws),
                      static_cast<hipStream_t>(stream));
}

extern "C" vdbc_status vdbc_conv3x3_wgrad(const uint16_t* a, uint32_t ca, const uint16_t* b, uint32_t cb,
                                          uint32_t upsample, uint32_t n, uint32_t hs, uint32_t ws_, uint32_t stride,
                                          const uint16_t* dz, uint32_t coutp, uint32_t cout, float* dw, float* db,
                                          void* ws, uint64_t ws_bytes, void* stream)
{
    clear_error();
    if (!a || !dz || !dw || !db || !ws || (cb && !b)) return fail(VDBC_E_INVALID, "null argument");
    if (ca % 8 || cb % 8 || ca + cb == 0 || ca + cb > 64 || coutp % 8 || coutp < cout || coutp > 64 || cout == 0 ||
        (stride != 1 && stride != 2))
        return fail(VDBC_E_INVALID, "bad channel counts or stride");
    ConvIn in{a, b, (int)ca, (int)cb, (int)(upsample != 0), (int)n, (int)hs, (int)ws_};
    const uint64_t need = al(64ull * 9 * 64 * 2) + al(wgrad_partial_floats(in, (int)stride, (int)cout) * 4);
    if (ws_bytes < need) return fail(VDBC_E_BUFFER_TOO_SMALL, "workspace needs %llu bytes", (unsigned long long)need);
    if (!aligned16(a) || !aligned16(b) || !aligned16(dz)) return fail(VDBC_E_INVALID, "operands must be 16-byte aligned");
    float* part = reinterpret_cast<float*>(static_cast<uint8_t*>(ws) + al(64ull * 9 * 64 * 2));
    return conv_wgrad(in, (int)stride, dz, (int)coutp, (int)cout, dw, db, part, wgrad_partial_floats(in, (int)stride, (int)cout),
                      static_cast<hipStream_t>(stream));
}
