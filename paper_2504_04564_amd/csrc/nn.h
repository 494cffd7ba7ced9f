// Shapes of the learned denoiser (host + device).  The network is this
// project's own addition to the method: a 6-layer 3x3 convolutional U-Net,
// NHWC tensors, BF16 weights and activations, FP32 accumulation.
//
//   c1 = relu(conv(x, 8 -> 32))                     full resolution
//   c2 = relu(conv(c1, 32 -> 64, stride 2))         half
//   c3 = relu(conv(c2, 64 -> 64))                   half
//   c4 = relu(conv(nearest_up2(c3), 64 -> 32))      full
//   c5 = relu(conv(concat(c1, c4), 64 -> 32))       full
//   out = x.rgb + conv(c5, 32 -> 3)                 full, FP32
//
// x has 8 channels: RGB of a low-sample-count render, first-scatter depth
// fraction, primary transmittance, three zeros.  Parameters are one flat
// FP32 vector: per layer W[co][ky][kx][ci] then b[co].
#pragma once
#include <cstdint>

namespace vdbc {
namespace nn {

struct Layer {
    int cin, cout, stride;
    bool relu;
};

constexpr int kLayers = 6;
constexpr Layer kNet[kLayers] = {
    {8, 32, 1, true}, {32, 64, 2, true}, {64, 64, 1, true},
    {64, 32, 1, true}, {64, 32, 1, true}, {32, 3, 1, false},
};

inline uint64_t weight_count(int l) { return (uint64_t)kNet[l].cout * 9 * kNet[l].cin; }
inline uint64_t weight_offset(int l)
{
    uint64_t off = 0;
    for (int i = 0; i < l; ++i) off += weight_count(i) + kNet[i].cout;
    return off;
}
inline uint64_t bias_offset(int l) { return weight_offset(l) + weight_count(l); }
inline uint64_t param_count() { return weight_offset(kLayers); }

}  // namespace nn
}  // namespace vdbc
