// Status reporting, header parsing and the host-side structural validator.
#include <cstring>

#include "common.h"
#include "format.h"
#include "host_header.h"

namespace vdbc {

static thread_local std::string g_last_error;

vdbc_status fail(vdbc_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

void clear_error() { g_last_error.clear(); }

template <class T>
static T get(const uint8_t* p, int off)
{
    T v;
    std::memcpy(&v, p + off, sizeof(T));
    return v;
}

vdbc_status parse_header(const void* header, uint64_t bytes, Header* out)
{
    const uint8_t* p = static_cast<const uint8_t*>(header);
    if (!p) return fail(VDBC_E_INVALID, "null header");
    if (bytes < kHeaderBytes) return fail(VDBC_E_FORMAT, "buffer smaller than its header");
    if (std::memcmp(p, "VDBC", 4) != 0) return fail(VDBC_E_FORMAT, "bad magic");
    if (get<uint32_t>(p, hdr::version) != kVersion) return fail(VDBC_E_FORMAT, "unsupported version");
    Header h;
    h.nx = get<uint32_t>(p, hdr::nx);
    h.ny = get<uint32_t>(p, hdr::ny);
    h.nz = get<uint32_t>(p, hdr::nz);
    h.background = get<float>(p, hdr::background);
    h.rate = get<float>(p, hdr::rate);
    h.metric = get<uint32_t>(p, hdr::metric);
    h.flags = get<uint32_t>(p, hdr::flags);
    h.layout = get<uint32_t>(p, hdr::layout);
    h.partial_fraction = get<float>(p, hdr::partial_fraction);
    h.partial_threshold = get<float>(p, hdr::partial_threshold);
    h.n_bricks = get<uint64_t>(p, hdr::n_bricks);
    h.k_bricks = get<uint64_t>(p, hdr::k_bricks);
    h.active_voxels = get<uint64_t>(p, hdr::active_voxels);
    h.n_upper = get<uint32_t>(p, hdr::n_upper);
    h.n_lower = get<uint32_t>(p, hdr::n_lower);
    h.n_leaf = get<uint32_t>(p, hdr::n_leaf);
    h.n_upper_tiles = get<uint32_t>(p, hdr::n_upper_tiles);
    h.n_lower_tiles = get<uint32_t>(p, hdr::n_lower_tiles);
    h.root_nx = get<uint32_t>(p, hdr::root_nx);
    h.root_ny = get<uint32_t>(p, hdr::root_ny);
    h.root_nz = get<uint32_t>(p, hdr::root_nz);
    h.off_root = get<uint64_t>(p, hdr::off_root);
    h.off_upper = get<uint64_t>(p, hdr::off_upper);
    h.off_lower = get<uint64_t>(p, hdr::off_lower);
    h.off_upper_tiles = get<uint64_t>(p, hdr::off_upper_tiles);
    h.off_lower_tiles = get<uint64_t>(p, hdr::off_lower_tiles);
    h.off_leaf_masks = get<uint64_t>(p, hdr::off_leaf_masks);
    h.off_leaf_values = get<uint64_t>(p, hdr::off_leaf_values);
    h.total_bytes = get<uint64_t>(p, hdr::total_bytes);
    if (h.layout >= kLayouts) return fail(VDBC_E_FORMAT, "unsupported layout %u", h.layout);
    if (h.nx == 0 || h.ny == 0 || h.nz == 0 || h.nx > 0x7FFFFFFFu || h.ny > 0x7FFFFFFFu ||
        h.nz > 0x7FFFFFFFu)
        return fail(VDBC_E_FORMAT, "bad dims");
    if (h.root_nx != (h.nx + 4095) / 4096 || h.root_ny != (h.ny + 4095) / 4096 ||
        h.root_nz != (h.nz + 4095) / 4096)
        return fail(VDBC_E_FORMAT, "root table does not match dims");
    uint64_t rn = (uint64_t)h.root_nx * h.root_ny * h.root_nz;
    // offsets must be exactly the canonical section layout
    uint64_t o = kHeaderBytes;
    if (h.off_root != o) return fail(VDBC_E_FORMAT, "bad root offset");
    o = align256(o + 4 * rn);
    if (h.off_upper != o) return fail(VDBC_E_FORMAT, "bad upper offset");
    o = align256(o + (uint64_t)h.n_upper * node_bytes(h.layout, kUpperWords));
    if (h.off_lower != o) return fail(VDBC_E_FORMAT, "bad lower offset");
    o = align256(o + (uint64_t)h.n_lower * node_bytes(h.layout, kLowerWords));
    if (h.off_upper_tiles != o) return fail(VDBC_E_FORMAT, "bad upper-tile offset");
    o = align256(o + 4ull * h.n_upper_tiles);
    if (h.off_lower_tiles != o) return fail(VDBC_E_FORMAT, "bad lower-tile offset");
    o = align256(o + 4ull * h.n_lower_tiles);
    if (h.off_leaf_masks != o) return fail(VDBC_E_FORMAT, "bad leaf-mask offset");
    o = align256(o + 64ull * h.n_leaf);
    if (h.off_leaf_values != o) return fail(VDBC_E_FORMAT, "bad leaf-value offset");
    o = align256(o + 2048ull * h.n_leaf);
    if (h.total_bytes != o) return fail(VDBC_E_FORMAT, "bad total size");
    if (h.total_bytes > bytes)
        return fail(VDBC_E_FORMAT, "buffer holds %llu bytes, header says %llu",
                    (unsigned long long)bytes, (unsigned long long)h.total_bytes);
    *out = h;
    return VDBC_OK;
}

static int popc(uint64_t x) { return __builtin_popcountll(x); }

// Walks every node record: running prefixes, totals, root entries.
static vdbc_status check_nodes(const uint8_t* p, const Header& h)
{
    uint64_t rn = (uint64_t)h.root_nx * h.root_ny * h.root_nz;
    const uint32_t* root = reinterpret_cast<const uint32_t*>(p + h.off_root);
    uint32_t expect_u = 0;
    for (uint64_t r = 0; r < rn; ++r) {
        if (root[r] == kNoChild) continue;
        if (root[r] != expect_u) return fail(VDBC_E_FORMAT, "root entries out of order");
        ++expect_u;
    }
    if (expect_u != h.n_upper) return fail(VDBC_E_FORMAT, "root references %u of %u uppers",
                                           expect_u, h.n_upper);
    struct Level {
        uint64_t off;
        uint32_t nodes, words, children, tiles;
    } levels[2] = {{h.off_upper, h.n_upper, kUpperWords, h.n_lower, h.n_upper_tiles},
                   {h.off_lower, h.n_lower, kLowerWords, h.n_leaf, h.n_lower_tiles}};
    const bool soa = (h.layout & kLayoutSoA) != 0;
    for (const Level& L : levels) {
        uint64_t c = 0, t = 0;
        for (uint64_t n = 0; n < L.nodes; ++n) {
            const uint8_t* node = p + L.off + n * node_bytes(h.layout, L.words);
            for (uint32_t i = 0; i < L.words; ++i) {
                NodeWord w;
                read_word(node, L.words, i, soa, &w);
                if (w.child_index != c || w.tile_index != t)
                    return fail(VDBC_E_FORMAT, "node %llu word %u: prefix mismatch", (unsigned long long)n, i);
                if (w.child & w.tile) return fail(VDBC_E_FORMAT, "slot both child and tile");
                if (w.reserved) return fail(VDBC_E_FORMAT, "reserved word not zero");
                c += popc(w.child);
                t += popc(w.tile);
            }
        }
        if (c != L.children || t != L.tiles)
            return fail(VDBC_E_FORMAT, "node masks count %llu children / %llu tiles",
                        (unsigned long long)c, (unsigned long long)t);
    }
    return VDBC_OK;
}

}  // namespace vdbc

using namespace vdbc;

extern "C" const char* vdbc_status_string(vdbc_status s)
{
    switch (s) {
    case VDBC_OK: return "ok";
    case VDBC_E_INVALID: return "invalid argument";
    case VDBC_E_NOMEM: return "out of memory";
    case VDBC_E_BUFFER_TOO_SMALL: return "buffer too small";
    case VDBC_E_FORMAT: return "bad buffer format";
    case VDBC_E_DEVICE: return "device error";
    case VDBC_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

extern "C" const char* vdbc_last_error(void) { return g_last_error.c_str(); }

extern "C" uint32_t vdbc_abi_version(void) { return VDBC_ABI_VERSION; }

#ifndef VDBC_SOURCE_HASH
#define VDBC_SOURCE_HASH "unknown"
#endif
extern "C" const char* vdbc_source_hash(void) { return VDBC_SOURCE_HASH; }

extern "C" vdbc_status vdbc_validate(const void* buf, uint64_t bytes, vdbc_encode_stats* info)
{
    clear_error();
    Header h;
    vdbc_status s = parse_header(buf, bytes, &h);
    if (s) return s;
    s = check_nodes(static_cast<const uint8_t*>(buf), h);
    if (s) return s;
    if (info) {
        info->background = h.background;
        info->n_bricks = h.n_bricks;
        info->k_bricks = h.k_bricks;
        info->n_leaf = h.n_leaf;
        info->n_lower = h.n_lower;
        info->n_upper = h.n_upper;
        info->n_lower_tiles = h.n_lower_tiles;
        info->n_upper_tiles = h.n_upper_tiles;
        info->active_voxels = h.active_voxels;
        info->bytes = h.total_bytes;
        info->achieved_rate = (double)h.active_voxels / ((double)h.nx * h.ny * h.nz);
    }
    return VDBC_OK;
}

extern "C" vdbc_status vdbc_grid_init(vdbc_grid* g, const void* device, uint64_t bytes,
                                      const void* host_header)
{
    clear_error();
    if (!g || !device || !host_header) return fail(VDBC_E_INVALID, "vdbc_grid_init: null argument");
    if (reinterpret_cast<uintptr_t>(device) % 256 != 0)
        return fail(VDBC_E_INVALID, "vdbc_grid_init: device buffer not 256-byte aligned");
    Header h;
    vdbc_status s = parse_header(host_header, bytes, &h);
    if (s) return s;
    if (h.layout != 0)
        return fail(VDBC_E_UNSUPPORTED, "vdbc_grid_init: the device kernels read node layout 0 only (buffer has %u)",
                    h.layout);
    g->device = device;
    g->bytes = bytes;
    std::memcpy(g->header, host_header, kHeaderBytes);
    return VDBC_OK;
}
