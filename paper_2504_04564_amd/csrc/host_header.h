// Host-side buffer helpers shared by the API, the layout converter and the
// launchers: header parsing, node words of either record layout, slot numbers.
#pragma once
#include <cstring>

#include "common.h"
#include "format.h"

namespace vdbc {
// Parses and checks the 256-byte header of a buffer of `bytes` bytes
// (canonical section layout for its node layout, dims, root table shape).
vdbc_status parse_header(const void* header, uint64_t bytes, Header* out);

// One word of a node, unpacked.
struct NodeWord {
    uint64_t child = 0, tile = 0, reserved = 0;
    uint32_t child_index = 0, tile_index = 0;
};

// Word i of a node of `words` words, records (soa = false) or four arrays.
inline void read_word(const uint8_t* node, uint32_t words, uint32_t i, bool soa, NodeWord* w)
{
    if (soa) {
        std::memcpy(&w->child, node + 8ull * i, 8);
        std::memcpy(&w->tile, node + 8ull * (words + i), 8);
        std::memcpy(&w->child_index, node + 16ull * words + 4ull * i, 4);
        std::memcpy(&w->tile_index, node + 20ull * words + 4ull * i, 4);
        w->reserved = 0;
        return;
    }
    Word r;
    std::memcpy(&r, node + 32ull * i, sizeof(Word));
    w->child = r.child;
    w->tile = r.tile;
    w->reserved = r.reserved;
    w->child_index = r.child_index;
    w->tile_index = r.tile_index;
}

inline void write_word(uint8_t* node, uint32_t words, uint32_t i, bool soa, const NodeWord& w)
{
    if (soa) {
        std::memcpy(node + 8ull * i, &w.child, 8);
        std::memcpy(node + 8ull * (words + i), &w.tile, 8);
        std::memcpy(node + 16ull * words + 4ull * i, &w.child_index, 4);
        std::memcpy(node + 20ull * words + 4ull * i, &w.tile_index, 4);
        return;
    }
    Word r{w.child, w.child_index, w.tile_index, w.tile, 0};
    std::memcpy(node + 32ull * i, &r, sizeof(Word));
}

// Slot number of child (x, y, z) (each < 2^log2) of a node: x-fastest, or
// with kLayoutMorton bit 3b+a of the number = bit b of coordinate a.
inline uint32_t slot_of(uint32_t layout, uint32_t log2, uint32_t x, uint32_t y, uint32_t z)
{
    if (!(layout & kLayoutMorton)) return x + ((y + (z << log2)) << log2);
    uint32_t n = 0;
    for (uint32_t b = 0; b < log2; ++b)
        n |= (((x >> b) & 1u) << (3 * b)) | (((y >> b) & 1u) << (3 * b + 1)) | (((z >> b) & 1u) << (3 * b + 2));
    return n;
}

inline void coords_of(uint32_t layout, uint32_t log2, uint32_t n, uint32_t* x, uint32_t* y, uint32_t* z)
{
    const uint32_t m = (1u << log2) - 1u;
    if (!(layout & kLayoutMorton)) {
        *x = n & m;
        *y = (n >> log2) & m;
        *z = n >> (2 * log2);
        return;
    }
    *x = *y = *z = 0;
    for (uint32_t b = 0; b < log2; ++b) {
        *x |= ((n >> (3 * b)) & 1u) << b;
        *y |= ((n >> (3 * b + 1)) & 1u) << b;
        *z |= ((n >> (3 * b + 2)) & 1u) << b;
    }
}

// Section offsets and total size for a header's counts and node layout.
inline void layout_sections(Header* h)
{
    const uint64_t rn = (uint64_t)h->root_nx * h->root_ny * h->root_nz;
    h->off_root = kHeaderBytes;
    h->off_upper = align256(h->off_root + 4 * rn);
    h->off_lower = align256(h->off_upper + (uint64_t)h->n_upper * node_bytes(h->layout, kUpperWords));
    h->off_upper_tiles = align256(h->off_lower + (uint64_t)h->n_lower * node_bytes(h->layout, kLowerWords));
    h->off_lower_tiles = align256(h->off_upper_tiles + 4ull * h->n_upper_tiles);
    h->off_leaf_masks = align256(h->off_lower_tiles + 4ull * h->n_lower_tiles);
    h->off_leaf_values = align256(h->off_leaf_masks + 64ull * h->n_leaf);
    h->total_bytes = align256(h->off_leaf_values + 2048ull * h->n_leaf);
}
}  // namespace vdbc
