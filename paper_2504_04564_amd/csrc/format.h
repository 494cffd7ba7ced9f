// Canonical buffer, format v1 (product side).
//
// The tree is the VDB of Section 3.2: 8^3-voxel leaves, lower internal nodes
// with 16^3 child slots (128^3 voxels), upper internal nodes with 32^3 child
// slots (4096^3 voxels), and a root table over ceil(dims/4096).  Each internal
// node is an array of 32-byte word records covering 64 slots each:
//
//   u64 child_mask   bit s set: slot 64*w+s holds a child node
//   u32 child_index  absolute index of the first child at or after slot 64*w
//   u32 tile_index   absolute index of the first tile at or after slot 64*w
//   u64 tile_mask    bit s set: slot holds an active constant tile
//   u64 reserved     zero
//
// so the first 16 bytes (one dwordx4 load) resolve the common child case and a
// child's index is child_index + popcount(child_mask & below(s)).  Sections:
// header 256 B | root u32[] | uppers | lowers | upper tiles f32[] | lower tiles
// f32[] | leaf masks u64[8] per leaf | leaf values f32[512] per leaf, each
// section 256-byte aligned; slots, leaf voxels and the root table x-fastest.
#pragma once
#include <cstdint>

namespace vdbc {

constexpr uint32_t kVersion = 1;
constexpr uint32_t kHeaderBytes = 256;
constexpr uint32_t kUpperWords = 512;   // 32^3 slots / 64
constexpr uint32_t kLowerWords = 64;    // 16^3 slots / 64
constexpr uint32_t kWordBytes = 32;
constexpr uint32_t kLeafVoxels = 512;
constexpr uint32_t kBrick = 32;
constexpr uint32_t kNoChild = 0xFFFFFFFFu;

struct alignas(16) Word {
    uint64_t child;
    uint32_t child_index;
    uint32_t tile_index;
    uint64_t tile;
    uint64_t reserved;
};
static_assert(sizeof(Word) == 32, "word record is 32 bytes");

// Header byte offsets.
namespace hdr {
constexpr int magic = 0, version = 4, nx = 8, ny = 12, nz = 16, background = 20, rate = 24,
              metric = 28, flags = 32, layout = 36, n_bricks = 40, k_bricks = 48,
              active_voxels = 56, n_upper = 64, n_lower = 68, n_leaf = 72,
              n_upper_tiles = 76, n_lower_tiles = 80, root_nx = 84, root_ny = 88,
              root_nz = 92, off_root = 96, off_upper = 104, off_lower = 112,
              off_upper_tiles = 120, off_lower_tiles = 128, off_leaf_masks = 136,
              off_leaf_values = 144, total_bytes = 152, partial_fraction = 160,
              partial_threshold = 164;
}

// Parsed header (host side).
struct Header {
    uint32_t nx, ny, nz;
    float background;
    float rate;
    uint32_t metric, flags, layout;
    float partial_fraction, partial_threshold;   // VDBC_PARTIAL only, else 0
    uint64_t n_bricks, k_bricks, active_voxels;
    uint32_t n_upper, n_lower, n_leaf, n_upper_tiles, n_lower_tiles;
    uint32_t root_nx, root_ny, root_nz;
    uint64_t off_root, off_upper, off_lower, off_upper_tiles, off_lower_tiles,
        off_leaf_masks, off_leaf_values, total_bytes;
};

inline uint64_t align256(uint64_t x) { return (x + 255u) & ~uint64_t(255u); }

// Node layouts (header field `layout`), two independent bits; 0 is the
// record layout above.
//   kLayoutMorton: the child slots of upper and lower nodes are numbered along
//     a Morton (Z-order) curve of the slot coordinates, bit 3b+a of the slot
//     number being bit b of coordinate a (x=0, y=1, z=2), instead of x-fastest.
//     Canonical order (children by slot) then stores lower nodes, leaves and
//     tiles along the curve, and one 64-slot word covers a 4^3 block of
//     children (for lower nodes: the 64 leaves of one 32^3 brick).
//   kLayoutSoA: a node of W words stores its fields as four arrays,
//     child masks u64[W] | tile masks u64[W] | child indices u32[W] | tile
//     indices u32[W], 24*W bytes, in place of W 32-byte records.
// Every layout holds the same tree: a lookup returns the same value.
constexpr uint32_t kLayoutMorton = 1;
constexpr uint32_t kLayoutSoA = 2;
constexpr uint32_t kLayouts = 4;
inline uint64_t node_bytes(uint32_t layout, uint32_t words)
{
    return ((layout & kLayoutSoA) ? 24ull : 32ull) * words;
}

}  // namespace vdbc
