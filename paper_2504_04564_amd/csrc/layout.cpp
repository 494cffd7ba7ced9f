// Node-layout conversion (host): rewrites a buffer into another node layout
// (x-fastest or Morton slot numbers, record or split-array node words) while
// keeping the tree of Section 3.2 unchanged.
//
// The destination follows the canonical order for its own slot numbering:
// uppers by root entry, lower nodes and upper tiles by (upper, slot), leaves
// and lower tiles by (lower, slot), every word's child and tile indices the
// running counts before it.  Leaf masks and values are copied unchanged, so
// only their order can differ.
#include <algorithm>
#include <cstring>
#include <vector>

#include "common.h"
#include "format.h"
#include "host_header.h"

namespace vdbc {
namespace {

template <class T>
T get(const uint8_t* p, uint64_t off)
{
    T v;
    std::memcpy(&v, p + off, sizeof(T));
    return v;
}

template <class T>
void put(uint8_t* p, uint64_t off, T v)
{
    std::memcpy(p + off, &v, sizeof(T));
}

// A child or tile of a node, keyed by its slot number in the destination.
struct Entry {
    uint32_t dst_slot;
    uint32_t is_child;
    uint32_t src_index;   // source lower / leaf index, or source tile index
};

// Children and tiles of one source node, in destination slot order.
void gather(const uint8_t* node, uint32_t words, uint32_t log2, uint32_t src_layout, uint32_t dst_layout,
            std::vector<Entry>* out)
{
    out->clear();
    const bool soa = (src_layout & kLayoutSoA) != 0;
    for (uint32_t w = 0; w < words; ++w) {
        NodeWord nw;
        read_word(node, words, w, soa, &nw);
        uint64_t both = nw.child | nw.tile;
        while (both) {
            const uint32_t bit = (uint32_t)__builtin_ctzll(both);
            both &= both - 1;
            const uint64_t below = (uint64_t(1) << bit) - 1u;
            uint32_t x, y, z;
            coords_of(src_layout, log2, 64u * w + bit, &x, &y, &z);
            Entry e;
            e.dst_slot = slot_of(dst_layout, log2, x, y, z);
            e.is_child = (uint32_t)((nw.child >> bit) & 1u);
            e.src_index = e.is_child ? nw.child_index + (uint32_t)__builtin_popcountll(nw.child & below)
                                     : nw.tile_index + (uint32_t)__builtin_popcountll(nw.tile & below);
            out->push_back(e);
        }
    }
    std::sort(out->begin(), out->end(), [](const Entry& a, const Entry& b) { return a.dst_slot < b.dst_slot; });
}

// Writes one destination node from its entries; `on_child` numbers a child
// (and emits its subtree), `on_tile` copies a tile value; both return the
// destination index.
template <class OnChild, class OnTile>
void emit(uint8_t* node, uint32_t words, bool soa, const std::vector<Entry>& es, uint32_t* child_count,
          uint32_t* tile_count, OnChild on_child, OnTile on_tile)
{
    size_t k = 0;
    for (uint32_t w = 0; w < words; ++w) {
        NodeWord nw;
        nw.child_index = *child_count;
        nw.tile_index = *tile_count;
        for (; k < es.size() && (es[k].dst_slot >> 6) == w; ++k) {
            const uint64_t bit = uint64_t(1) << (es[k].dst_slot & 63u);
            if (es[k].is_child) {
                nw.child |= bit;
                on_child(es[k].src_index);
                ++*child_count;
            } else {
                nw.tile |= bit;
                on_tile(es[k].src_index);
                ++*tile_count;
            }
        }
        write_word(node, words, w, soa, nw);
    }
}

}  // namespace
}  // namespace vdbc

using namespace vdbc;

extern "C" vdbc_status vdbc_relayout(const void* src_v, uint64_t src_bytes, uint32_t layout, void* out_v,
                                     uint64_t capacity, uint64_t* bytes)
{
    if (!src_v || !bytes) {
        clear_error();
        return fail(VDBC_E_INVALID, "vdbc_relayout: null argument");
    }
    vdbc_status s = vdbc_validate(src_v, src_bytes, nullptr);   // walks only consistent trees
    if (s) return s;
    if (layout >= kLayouts) return fail(VDBC_E_INVALID, "vdbc_relayout: layout must be 0..%u", kLayouts - 1);
    const uint8_t* src = static_cast<const uint8_t*>(src_v);
    Header sh;
    if ((s = parse_header(src, src_bytes, &sh))) return s;
    Header dh = sh;
    dh.layout = layout;
    layout_sections(&dh);
    *bytes = dh.total_bytes;
    if (!out_v || capacity < dh.total_bytes)
        return fail(VDBC_E_BUFFER_TOO_SMALL, "vdbc_relayout: need %llu bytes", (unsigned long long)dh.total_bytes);
    uint8_t* out = static_cast<uint8_t*>(out_v);
    if (out < src + sh.total_bytes && src < out + dh.total_bytes)
        return fail(VDBC_E_INVALID, "vdbc_relayout: source and destination overlap");
    try {
        std::memset(out, 0, dh.off_leaf_values);
        std::memcpy(out, src, kHeaderBytes);
        put<uint32_t>(out, hdr::layout, dh.layout);
        put<uint64_t>(out, hdr::off_root, dh.off_root);
        put<uint64_t>(out, hdr::off_upper, dh.off_upper);
        put<uint64_t>(out, hdr::off_lower, dh.off_lower);
        put<uint64_t>(out, hdr::off_upper_tiles, dh.off_upper_tiles);
        put<uint64_t>(out, hdr::off_lower_tiles, dh.off_lower_tiles);
        put<uint64_t>(out, hdr::off_leaf_masks, dh.off_leaf_masks);
        put<uint64_t>(out, hdr::off_leaf_values, dh.off_leaf_values);
        put<uint64_t>(out, hdr::total_bytes, dh.total_bytes);
        const uint64_t rn = (uint64_t)sh.root_nx * sh.root_ny * sh.root_nz;
        std::memcpy(out + dh.off_root, src + sh.off_root, 4 * rn);   // uppers keep their root order

        const bool dsoa = (layout & kLayoutSoA) != 0;
        const uint64_t su_bytes = node_bytes(sh.layout, kUpperWords), sl_bytes = node_bytes(sh.layout, kLowerWords);
        const uint64_t du_bytes = node_bytes(layout, kUpperWords), dl_bytes = node_bytes(layout, kLowerWords);
        uint32_t lower_i = 0, leaf_i = 0, utile_i = 0, ltile_i = 0;
        std::vector<Entry> ue, le;
        for (uint32_t u = 0; u < sh.n_upper; ++u) {
            gather(src + sh.off_upper + u * su_bytes, kUpperWords, 5, sh.layout, layout, &ue);
            auto lower_child = [&](uint32_t sl) {
                uint8_t* dnode = out + dh.off_lower + (uint64_t)lower_i * dl_bytes;
                gather(src + sh.off_lower + (uint64_t)sl * sl_bytes, kLowerWords, 4, sh.layout, layout, &le);
                uint32_t child_next = leaf_i, tile_next = ltile_i;
                emit(
                    dnode, kLowerWords, dsoa, le, &child_next, &tile_next,
                    [&](uint32_t sf) {
                        std::memcpy(out + dh.off_leaf_masks + 64ull * child_next,
                                    src + sh.off_leaf_masks + 64ull * sf, 64);
                        std::memcpy(out + dh.off_leaf_values + 2048ull * child_next,
                                    src + sh.off_leaf_values + 2048ull * sf, 2048);
                    },
                    [&](uint32_t st) {
                        std::memcpy(out + dh.off_lower_tiles + 4ull * tile_next,
                                    src + sh.off_lower_tiles + 4ull * st, 4);
                    });
                leaf_i = child_next;
                ltile_i = tile_next;
            };
            uint32_t lower_next = lower_i, utile_next = utile_i;
            // a lower node's subtree is emitted when its slot is reached, so
            // lower_i must advance with the node counter of this upper
            emit(
                out + dh.off_upper + (uint64_t)u * du_bytes, kUpperWords, dsoa, ue, &lower_next, &utile_next,
                [&](uint32_t sl) {
                    lower_child(sl);
                    ++lower_i;
                },
                [&](uint32_t st) {
                    std::memcpy(out + dh.off_upper_tiles + 4ull * utile_i, src + sh.off_upper_tiles + 4ull * st, 4);
                    ++utile_i;
                });
        }
        const uint64_t end = dh.off_leaf_values + 2048ull * dh.n_leaf;
        std::memset(out + end, 0, dh.total_bytes - end);
        if (lower_i != dh.n_lower || leaf_i != dh.n_leaf || utile_i != dh.n_upper_tiles ||
            ltile_i != dh.n_lower_tiles)
            return fail(VDBC_E_FORMAT, "vdbc_relayout: node counts do not match the header");
    } catch (const std::bad_alloc&) {
        return fail(VDBC_E_NOMEM, "vdbc_relayout: out of host memory");
    }
    return VDBC_OK;
}
