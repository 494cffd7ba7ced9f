// Host encoder: Alg. 1 "Compress" (Section 3.1) and the VDB tree build +
// linearisation of Section 3.2, multithreaded and without any per-voxel side
// array (the paper-scale volume is 26 GB of float32).
//
// Steps, in the paper's order:
//   1. background B = value of the most populated histogram entry; here the
//      exact mode of the float values (-0 counted as +0, ties to the smallest
//      value), found with a 16-bit radix histogram fused with step 2, exact
//      counts inside the candidate buckets, and a sort fallback when the data
//      has no dominant value;
//   2. value range [lo, hi] of every 32^3 brick (partial edge bricks
//      included);
//   3. similarity f (Eq. 1-3) in double, bricks sorted by f descending (most
//      dissimilar from B first), ties by brick index;
//   4. activation of all voxels of the first K = min(N, floor(q*N + 0.5))
//      bricks plus the two extreme corner voxels (Section 3.2.1) — or, with
//      VDBC_PARTIAL, the partial-brick variant Section 3.2.1 leaves as future
//      work: bricks ranked below the similarity threshold share the same
//      voxel budget as a fraction of each brick (rule in vdbc.h), then
//      pruning at tolerance 0 (Section 3.2.1 tree.prune()): full uniform
//      leaves become lower-node tiles, lower nodes made of one uniform tile
//      value become upper-node tiles;
//   5. linearisation into the canonical buffer (format.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>

#include "common.h"
#include "format.h"

using namespace vdbc;

namespace {

inline uint32_t fbits(float v)
{
    uint32_t b;
    std::memcpy(&b, &v, 4);
    return b;
}

// Order-preserving key of a finite float, -0 folded onto +0.
inline uint32_t order_key(uint32_t b)
{
    if (b == 0x80000000u) b = 0;
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
inline float key_value(uint32_t k)
{
    uint32_t b = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
    float v;
    std::memcpy(&v, &b, 4);
    return v;
}

inline uint32_t cdiv(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

struct LeafRec {
    uint64_t key;       // root index << 27 | n1 << 12 | n2 (canonical order)
    uint32_t lx, ly, lz;
    uint32_t tile_bits; // valid if is_tile
    uint8_t in_brick;   // inside a selected brick (all in-volume voxels active)
    uint8_t is_tile;
    uint32_t part;      // index of its partially active brick, or kNoChild
};

// A partially active brick: its active voxels are those that come first in
// the order (|value - B| descending, linear index ascending), up to and
// including the last one taken, (d_last, i_last).
struct PartialBrick {
    uint32_t brick;
    uint64_t count;     // active voxels
    double d_last;
    uint64_t i_last;
    uint64_t leaf_any;  // bit l: leaf l (x-fastest 4^3 of the brick) holds an active voxel
};

struct LowerRec {
    uint64_t key;       // root index << 15 | n1
    uint32_t first, count;  // leaf range in the sorted leaf list
    uint32_t tile_bits;
    uint8_t is_tile;    // pruned into an upper tile
};

}  // namespace

struct vdbc_encoder {
    const float* dense = nullptr;
    uint32_t nx = 0, ny = 0, nz = 0;
    vdbc_encode_params p{};
    unsigned threads = 1;
    float B = 0.0f;
    uint64_t N = 0, K = 0;
    uint32_t nbx = 0, nby = 0, nbz = 0;
    std::vector<uint8_t> brick_sel;
    std::vector<PartialBrick> partial;
    std::vector<uint32_t> brick_part;  // brick -> index in `partial` or kNoChild
    std::vector<LeafRec> leaves;      // sorted by key
    std::vector<LowerRec> lowers;     // sorted by key
    std::vector<uint64_t> upper_root; // root index of each upper, ascending
    uint32_t rnx = 0, rny = 0, rnz = 0;
    uint64_t n_leaf = 0, n_lower = 0, n_upper = 0, n_ltile = 0, n_utile = 0;
    uint64_t active = 0;
    Header h{};
};

namespace {

uint64_t voxel_index(const vdbc_encoder& e, uint64_t x, uint64_t y, uint64_t z)
{
    return x + e.nx * (y + (uint64_t)e.ny * z);
}

// ---------------------------------------------------------------- step 1+2
vdbc_status scan_ranges_and_histogram(vdbc_encoder& e, std::vector<float>& lo,
                                      std::vector<float>& hi, std::vector<uint64_t>& hist)
{
    const uint64_t rows = (uint64_t)e.nby * e.nbz;
    std::vector<std::vector<uint64_t>> hists(e.threads);
    std::atomic<int> bad{0};
    const bool need_hist = !(e.p.flags & VDBC_BG_EXPLICIT);
    parallel_for(rows, e.threads, [&](uint64_t row, unsigned t) {
        if (need_hist && hists[t].empty()) hists[t].assign(65536, 0);
        uint64_t* H = need_hist ? hists[t].data() : nullptr;
        uint32_t by = (uint32_t)(row % e.nby), bz = (uint32_t)(row / e.nby);
        uint64_t base = (uint64_t)e.nbx * (by + (uint64_t)e.nby * bz);
        std::vector<float> l(e.nbx, INFINITY), h(e.nbx, -INFINITY);
        int nonfinite = 0;
        for (uint32_t z = bz * kBrick; z < e.nz && z < (bz + 1) * kBrick; ++z)
            for (uint32_t y = by * kBrick; y < e.ny && y < (by + 1) * kBrick; ++y) {
                const float* r = e.dense + voxel_index(e, 0, y, z);
                for (uint32_t bx = 0; bx < e.nbx; ++bx) {
                    uint32_t x0 = bx * kBrick, x1 = std::min(e.nx, x0 + kBrick);
                    float mn = l[bx], mx = h[bx];
                    for (uint32_t x = x0; x < x1; ++x) {
                        float v = r[x];
                        uint32_t b = fbits(v);
                        nonfinite |= ((b & 0x7F800000u) == 0x7F800000u);
                        mn = v < mn ? v : mn;
                        mx = v > mx ? v : mx;
                        if (H) ++H[order_key(b) >> 16];
                    }
                    l[bx] = mn;
                    h[bx] = mx;
                }
            }
        if (nonfinite) bad.store(1);
        for (uint32_t bx = 0; bx < e.nbx; ++bx) {
            lo[base + bx] = l[bx];
            hi[base + bx] = h[bx];
        }
    });
    if (bad.load()) return fail(VDBC_E_INVALID, "vdbc_encode: input holds NaN or Inf");
    if (need_hist) {
        hist.assign(65536, 0);
        for (auto& H : hists)
            if (!H.empty())
                for (int i = 0; i < 65536; ++i) hist[i] += H[i];
    }
    return VDBC_OK;
}

// Exact counts of the values inside a batch of 16-bit buckets.
void count_buckets(const vdbc_encoder& e, const std::vector<uint32_t>& buckets,
                   std::vector<uint64_t>& counts)
{
    const uint64_t n = (uint64_t)e.nx * e.ny * e.nz;
    std::vector<int16_t> slot(65536, -1);
    for (size_t i = 0; i < buckets.size(); ++i) slot[buckets[i]] = (int16_t)i;
    const uint64_t chunk = 1u << 22;
    const uint64_t tasks = (n + chunk - 1) / chunk;
    std::vector<std::vector<uint32_t>> local(e.threads);
    parallel_for(tasks, e.threads, [&](uint64_t task, unsigned t) {
        if (local[t].empty()) local[t].assign(buckets.size() * 65536, 0);
        uint32_t* L = local[t].data();
        uint64_t a = task * chunk, b = std::min(n, a + chunk);
        for (uint64_t i = a; i < b; ++i) {
            uint32_t k = order_key(fbits(e.dense[i]));
            int s = slot[k >> 16];
            if (s >= 0) ++L[(uint64_t)s * 65536 + (k & 0xFFFFu)];
        }
    });
    counts.assign(buckets.size() * 65536, 0);
    for (auto& L : local)
        if (!L.empty())
            for (size_t i = 0; i < counts.size(); ++i) counts[i] += L[i];
}

// Sort fallback: exact mode over all keys.
vdbc_status mode_by_sort(const vdbc_encoder& e, float* out)
{
    const uint64_t n = (uint64_t)e.nx * e.ny * e.nz;
    std::unique_ptr<uint32_t[]> keys(new (std::nothrow) uint32_t[n]);
    if (!keys) return fail(VDBC_E_NOMEM, "vdbc_encode: no memory for the background sort");
    const unsigned T = e.threads;
    std::vector<uint64_t> bounds(T + 1);
    for (unsigned t = 0; t <= T; ++t) bounds[t] = n * t / T;
    parallel_for(T, T, [&](uint64_t t, unsigned) {
        for (uint64_t i = bounds[t]; i < bounds[t + 1]; ++i)
            keys[i] = order_key(fbits(e.dense[i]));
        std::sort(keys.get() + bounds[t], keys.get() + bounds[t + 1]);
    });
    for (uint64_t width = 1; width < T; width *= 2) {
        std::vector<uint64_t> starts;
        for (uint64_t t = 0; t + width < T; t += 2 * width) starts.push_back(t);
        parallel_for(starts.size(), T, [&](uint64_t s, unsigned) {
            uint64_t t = starts[s];
            uint64_t a = bounds[t], m = bounds[t + width],
                     b = bounds[std::min<uint64_t>(T, t + 2 * width)];
            std::inplace_merge(keys.get() + a, keys.get() + m, keys.get() + b);
        });
    }
    uint64_t best = 0;
    uint32_t best_key = keys[0];
    for (uint64_t i = 0; i < n;) {
        uint64_t j = i;
        while (j < n && keys[j] == keys[i]) ++j;
        if (j - i > best) {
            best = j - i;
            best_key = keys[i];
        }
        i = j;
    }
    *out = key_value(best_key);
    return VDBC_OK;
}

vdbc_status background_mode(vdbc_encoder& e, const std::vector<uint64_t>& hist)
{
    std::vector<uint32_t> order;
    for (uint32_t b = 0; b < 65536; ++b)
        if (hist[b]) order.push_back(b);
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t b) { return hist[a] > hist[b]; });
    uint64_t best = 0;
    uint32_t best_key = 0xFFFFFFFFu;
    size_t pos = 0;
    const size_t batch = 8, max_batches = 4;
    for (size_t round = 0; pos < order.size() && hist[order[pos]] >= best; ++round) {
        if (round == max_batches) {
            // no dominant value: exact counting by sorting every key
            return mode_by_sort(e, &e.B);
        }
        std::vector<uint32_t> bk;
        while (pos < order.size() && bk.size() < batch && hist[order[pos]] >= best)
            bk.push_back(order[pos++]);
        std::vector<uint64_t> counts;
        count_buckets(e, bk, counts);
        for (size_t s = 0; s < bk.size(); ++s)
            for (uint32_t lo = 0; lo < 65536; ++lo) {
                uint64_t c = counts[s * 65536 + lo];
                if (!c) continue;
                uint32_t k = (bk[s] << 16) | lo;
                if (c > best || (c == best && k < best_key)) {
                    best = c;
                    best_key = k;
                }
            }
    }
    e.B = key_value(best_key);
    return VDBC_OK;
}

// ---------------------------------------------------------------- step 3+4
uint32_t leaf_extent(uint32_t l, uint32_t n) { return std::min<uint32_t>(8, n - 8 * l); }

bool is_corner(const vdbc_encoder& e, uint64_t x, uint64_t y, uint64_t z)
{
    if (e.p.flags & VDBC_NO_CORNERS) return false;
    return (x == 0 && y == 0 && z == 0) || (x == e.nx - 1u && y == e.ny - 1u && z == e.nz - 1u);
}

uint64_t brick_voxels(const vdbc_encoder& e, uint32_t b)
{
    uint32_t bx = b % e.nbx, by = (b / e.nbx) % e.nby, bz = b / (e.nbx * e.nby);
    return (uint64_t)std::min(kBrick, e.nx - bx * kBrick) * std::min(kBrick, e.ny - by * kBrick) *
           std::min(kBrick, e.nz - bz * kBrick);
}

// Voxel (x, y, z) of partially active brick P is active.
inline bool partial_active(const vdbc_encoder& e, const PartialBrick& P, uint64_t x, uint64_t y,
                           uint64_t z)
{
    const uint64_t i = voxel_index(e, x, y, z);
    const double d = std::fabs((double)e.dense[i] - (double)e.B);
    return d > P.d_last || (d == P.d_last && i <= P.i_last);
}

// The voxel active in brick-selection terms (full brick, partial brick or
// corner), for a leaf record.
inline bool leaf_voxel_active(const vdbc_encoder& e, const LeafRec& L, uint64_t x, uint64_t y,
                              uint64_t z)
{
    if (L.in_brick || is_corner(e, x, y, z)) return true;
    return L.part != kNoChild && partial_active(e, e.partial[L.part], x, y, z);
}

// Partial-brick activation: the counts per brick from the budget walk, the
// last voxel taken in each partially active brick and its leaf occupancy.
// Bricks that end up with all their voxels join `selected`.
vdbc_status plan_partial(vdbc_encoder& e, const std::vector<uint32_t>& order, uint64_t F,
                         std::vector<uint32_t>& selected)
{
    uint64_t R = 0;
    for (uint64_t r = F; r < e.K; ++r) R += brick_voxels(e, order[r]);
    const double frac = (double)e.p.partial_fraction;
    std::vector<uint64_t> cnt(e.N - F, 0);
    for (int sweep = 0; sweep < 2 && R > 0; ++sweep)
        for (uint64_t r = F; r < e.N && R > 0; ++r) {
            const uint64_t v = brick_voxels(e, order[r]);
            const uint64_t share = std::min<uint64_t>(v, (uint64_t)std::ceil(frac * (double)v));
            const uint64_t want = sweep == 0 ? share : v - share;
            const uint64_t take = std::min(want, R);
            cnt[r - F] += take;
            R -= take;
        }
    e.partial.clear();
    e.brick_part.assign(e.N, kNoChild);
    for (uint64_t r = F; r < e.N; ++r) {
        const uint64_t c = cnt[r - F];
        if (c == 0) continue;
        if (c == brick_voxels(e, order[r])) {
            selected.push_back(order[r]);
            continue;
        }
        e.brick_part[order[r]] = (uint32_t)e.partial.size();
        e.partial.push_back(PartialBrick{order[r], c, 0.0, 0, 0});
    }
    struct Key {
        double d;
        uint64_t i;
    };
    std::vector<std::vector<Key>> scratch(e.threads);
    parallel_for(e.partial.size(), e.threads, [&](uint64_t pi, unsigned t) {
        PartialBrick& P = e.partial[pi];
        const uint32_t bx = P.brick % e.nbx, by = (P.brick / e.nbx) % e.nby, bz = P.brick / (e.nbx * e.nby);
        std::vector<Key>& k = scratch[t];
        k.clear();
        for (uint32_t z = bz * kBrick; z < e.nz && z < (bz + 1) * kBrick; ++z)
            for (uint32_t y = by * kBrick; y < e.ny && y < (by + 1) * kBrick; ++y)
                for (uint32_t x = bx * kBrick; x < e.nx && x < (bx + 1) * kBrick; ++x) {
                    const uint64_t i = voxel_index(e, x, y, z);
                    k.push_back(Key{std::fabs((double)e.dense[i] - (double)e.B), i});
                }
        auto before = [](const Key& a, const Key& b) { return a.d > b.d || (a.d == b.d && a.i < b.i); };
        std::nth_element(k.begin(), k.begin() + (P.count - 1), k.end(), before);
        P.d_last = k[P.count - 1].d;
        P.i_last = k[P.count - 1].i;
        uint64_t any = 0;
        for (uint32_t z = bz * kBrick; z < e.nz && z < (bz + 1) * kBrick; ++z)
            for (uint32_t y = by * kBrick; y < e.ny && y < (by + 1) * kBrick; ++y)
                for (uint32_t x = bx * kBrick; x < e.nx && x < (bx + 1) * kBrick; ++x)
                    if (partial_active(e, P, x, y, z)) {
                        const uint32_t l = ((x >> 3) & 3) + 4 * (((y >> 3) & 3) + 4 * ((z >> 3) & 3));
                        any |= uint64_t(1) << l;
                    }
        P.leaf_any = any;
    });
    return VDBC_OK;
}

vdbc_status build_tree(vdbc_encoder& e, const std::vector<uint32_t>& selected)
{
    const bool prune = !(e.p.flags & VDBC_NO_PRUNE);
    const uint32_t lgx = cdiv(e.nx, 8), lgy = cdiv(e.ny, 8), lgz = cdiv(e.nz, 8);
    e.rnx = cdiv(e.nx, 4096);
    e.rny = cdiv(e.ny, 4096);
    e.rnz = cdiv(e.nz, 4096);
    auto make_key = [&](uint32_t lx, uint32_t ly, uint32_t lz) {
        uint64_t Lx = lx >> 4, Ly = ly >> 4, Lz = lz >> 4;
        uint64_t r = (Lx >> 5) + e.rnx * ((Ly >> 5) + (uint64_t)e.rny * (Lz >> 5));
        uint64_t n1 = (Lx & 31) + 32 * ((Ly & 31) + 32 * (Lz & 31));
        uint64_t n2 = (lx & 15) + 16 * ((ly & 15) + 16 * (lz & 15));
        return (r << 27) | (n1 << 12) | n2;
    };
    // leaves of the selected bricks
    e.leaves.clear();
    e.leaves.reserve(selected.size() * 64 + 2);
    for (uint32_t b : selected) {
        uint32_t bx = b % e.nbx, by = (b / e.nbx) % e.nby, bz = b / (e.nbx * e.nby);
        for (uint32_t k = 0; k < 4; ++k)
            for (uint32_t j = 0; j < 4; ++j)
                for (uint32_t i = 0; i < 4; ++i) {
                    uint32_t lx = 4 * bx + i, ly = 4 * by + j, lz = 4 * bz + k;
                    if (lx >= lgx || ly >= lgy || lz >= lgz) continue;
                    e.leaves.push_back(LeafRec{make_key(lx, ly, lz), lx, ly, lz, 0, 1, 0, kNoChild});
                }
    }
    // leaves of partially active bricks that hold an active voxel
    for (uint32_t pi = 0; pi < e.partial.size(); ++pi) {
        const PartialBrick& P = e.partial[pi];
        uint32_t bx = P.brick % e.nbx, by = (P.brick / e.nbx) % e.nby, bz = P.brick / (e.nbx * e.nby);
        for (uint32_t l = 0; l < 64; ++l)
            if (P.leaf_any >> l & 1) {
                uint32_t lx = 4 * bx + (l & 3), ly = 4 * by + ((l >> 2) & 3), lz = 4 * bz + (l >> 4);
                e.leaves.push_back(LeafRec{make_key(lx, ly, lz), lx, ly, lz, 0, 0, 0, pi});
            }
    }
    // corner leaves outside the selection
    if (!(e.p.flags & VDBC_NO_CORNERS)) {
        uint32_t cl[2][3] = {{0, 0, 0}, {(e.nx - 1) / 8, (e.ny - 1) / 8, (e.nz - 1) / 8}};
        for (int c = 0; c < 2; ++c) {
            uint32_t lx = cl[c][0], ly = cl[c][1], lz = cl[c][2];
            uint32_t b = (lx / 4) + e.nbx * ((ly / 4) + e.nby * (lz / 4));
            if (e.brick_sel[b]) continue;
            const uint32_t pi = e.partial.empty() ? kNoChild : e.brick_part[b];
            const uint32_t l = (lx & 3) + 4 * ((ly & 3) + 4 * (lz & 3));
            if (pi != kNoChild && (e.partial[pi].leaf_any >> l & 1)) continue;  // leaf exists
            if (c == 1 && lx == 0 && ly == 0 && lz == 0) continue;  // same leaf
            e.leaves.push_back(LeafRec{make_key(lx, ly, lz), lx, ly, lz, 0, 0, 0, pi});
        }
    }
    std::sort(e.leaves.begin(), e.leaves.end(),
              [](const LeafRec& a, const LeafRec& b) { return a.key < b.key; });
    // prune full uniform leaves (all 512 voxels in-volume and active)
    if (prune) {
        parallel_for(e.leaves.size(), e.threads, [&](uint64_t li, unsigned) {
            LeafRec& L = e.leaves[li];
            if (!L.in_brick && L.part == kNoChild) return;
            if (leaf_extent(L.lx, e.nx) != 8 || leaf_extent(L.ly, e.ny) != 8 ||
                leaf_extent(L.lz, e.nz) != 8)
                return;
            const uint32_t first = fbits(e.dense[voxel_index(e, 8u * L.lx, 8u * L.ly, 8u * L.lz)]);
            for (uint32_t k = 0; k < 8; ++k)
                for (uint32_t j = 0; j < 8; ++j) {
                    const float* r = e.dense + voxel_index(e, 8u * L.lx, 8u * L.ly + j, 8u * L.lz + k);
                    for (uint32_t i = 0; i < 8; ++i)
                        if (fbits(r[i]) != first) return;
                }
            // a leaf of a partially active brick is a tile only if all 512 are active
            if (!L.in_brick)
                for (uint32_t k = 0; k < 8; ++k)
                    for (uint32_t j = 0; j < 8; ++j)
                        for (uint32_t i = 0; i < 8; ++i)
                            if (!leaf_voxel_active(e, L, 8ull * L.lx + i, 8ull * L.ly + j, 8ull * L.lz + k))
                                return;
            L.is_tile = 1;
            L.tile_bits = first;
        });
    }
    // lower nodes = runs of equal (key >> 12)
    e.lowers.clear();
    for (uint32_t i = 0; i < e.leaves.size();) {
        uint32_t j = i;
        uint64_t lk = e.leaves[i].key >> 12;
        bool uniform = true;
        while (j < e.leaves.size() && (e.leaves[j].key >> 12) == lk) {
            if (!e.leaves[j].is_tile || e.leaves[j].tile_bits != e.leaves[i].tile_bits)
                uniform = false;
            ++j;
        }
        LowerRec L{lk, i, j - i, e.leaves[i].tile_bits, 0};
        if (prune && uniform && (j - i) == 4096) L.is_tile = 1;
        e.lowers.push_back(L);
        i = j;
    }
    // counts
    e.n_leaf = e.n_ltile = e.n_lower = e.n_utile = 0;
    for (const LowerRec& L : e.lowers) {
        if (L.is_tile) {
            ++e.n_utile;
            continue;
        }
        ++e.n_lower;
        for (uint32_t i = L.first; i < L.first + L.count; ++i) {
            if (e.leaves[i].is_tile) ++e.n_ltile;
            else ++e.n_leaf;
        }
    }
    e.upper_root.clear();
    for (const LowerRec& L : e.lowers) {
        uint64_t r = L.key >> 15;
        if (e.upper_root.empty() || e.upper_root.back() != r) e.upper_root.push_back(r);
    }
    e.n_upper = e.upper_root.size();
    if (e.n_leaf > 0xFFFFFFFFull || e.n_lower > 0xFFFFFFFFull)
        return fail(VDBC_E_UNSUPPORTED, "vdbc_encode: more than 2^32 leaves");
    return VDBC_OK;
}

void fill_header(vdbc_encoder& e)
{
    Header& h = e.h;
    h.nx = e.nx;
    h.ny = e.ny;
    h.nz = e.nz;
    h.background = e.B;
    h.rate = e.p.rate;
    h.metric = e.p.metric;
    h.flags = e.p.flags;
    h.partial_fraction = (e.p.flags & VDBC_PARTIAL) ? e.p.partial_fraction : 0.0f;
    h.partial_threshold = (e.p.flags & VDBC_PARTIAL) ? e.p.partial_threshold : 0.0f;
    h.layout = 0;
    h.n_bricks = e.N;
    h.k_bricks = e.K;
    h.active_voxels = e.active;
    h.n_upper = (uint32_t)e.n_upper;
    h.n_lower = (uint32_t)e.n_lower;
    h.n_leaf = (uint32_t)e.n_leaf;
    h.n_upper_tiles = (uint32_t)e.n_utile;
    h.n_lower_tiles = (uint32_t)e.n_ltile;
    h.root_nx = e.rnx;
    h.root_ny = e.rny;
    h.root_nz = e.rnz;
    uint64_t rn = (uint64_t)e.rnx * e.rny * e.rnz;
    h.off_root = kHeaderBytes;
    h.off_upper = align256(h.off_root + 4 * rn);
    h.off_lower = align256(h.off_upper + e.n_upper * kUpperWords * kWordBytes);
    h.off_upper_tiles = align256(h.off_lower + e.n_lower * kLowerWords * kWordBytes);
    h.off_lower_tiles = align256(h.off_upper_tiles + 4 * e.n_utile);
    h.off_leaf_masks = align256(h.off_lower_tiles + 4 * e.n_ltile);
    h.off_leaf_values = align256(h.off_leaf_masks + 64 * e.n_leaf);
    h.total_bytes = align256(h.off_leaf_values + 2048 * e.n_leaf);
}

template <class T>
void put(uint8_t* base, uint64_t off, T v)
{
    std::memcpy(base + off, &v, sizeof(T));
}

void write_header(const Header& h, uint8_t* o)
{
    std::memset(o, 0, kHeaderBytes);
    std::memcpy(o, "VDBC", 4);
    put<uint32_t>(o, hdr::version, kVersion);
    put<uint32_t>(o, hdr::nx, h.nx);
    put<uint32_t>(o, hdr::ny, h.ny);
    put<uint32_t>(o, hdr::nz, h.nz);
    put<float>(o, hdr::background, h.background);
    put<float>(o, hdr::rate, h.rate);
    put<uint32_t>(o, hdr::metric, h.metric);
    put<uint32_t>(o, hdr::flags, h.flags);
    put<uint32_t>(o, hdr::layout, h.layout);
    put<uint64_t>(o, hdr::n_bricks, h.n_bricks);
    put<uint64_t>(o, hdr::k_bricks, h.k_bricks);
    put<uint64_t>(o, hdr::active_voxels, h.active_voxels);
    put<uint32_t>(o, hdr::n_upper, h.n_upper);
    put<uint32_t>(o, hdr::n_lower, h.n_lower);
    put<uint32_t>(o, hdr::n_leaf, h.n_leaf);
    put<uint32_t>(o, hdr::n_upper_tiles, h.n_upper_tiles);
    put<uint32_t>(o, hdr::n_lower_tiles, h.n_lower_tiles);
    put<uint32_t>(o, hdr::root_nx, h.root_nx);
    put<uint32_t>(o, hdr::root_ny, h.root_ny);
    put<uint32_t>(o, hdr::root_nz, h.root_nz);
    put<uint64_t>(o, hdr::off_root, h.off_root);
    put<uint64_t>(o, hdr::off_upper, h.off_upper);
    put<uint64_t>(o, hdr::off_lower, h.off_lower);
    put<uint64_t>(o, hdr::off_upper_tiles, h.off_upper_tiles);
    put<uint64_t>(o, hdr::off_lower_tiles, h.off_lower_tiles);
    put<uint64_t>(o, hdr::off_leaf_masks, h.off_leaf_masks);
    put<uint64_t>(o, hdr::off_leaf_values, h.off_leaf_values);
    put<uint64_t>(o, hdr::total_bytes, h.total_bytes);
    if (h.flags & VDBC_PARTIAL) {
        put<float>(o, hdr::partial_fraction, h.partial_fraction);
        put<float>(o, hdr::partial_threshold, h.partial_threshold);
    }
}

}  // namespace

// ---------------------------------------------------------------- public API

extern "C" vdbc_status vdbc_encode_begin(const float* dense, vdbc_dims dims,
                                         const vdbc_encode_params* p, vdbc_encoder** out,
                                         uint64_t* bytes, vdbc_encode_stats* stats)
{
    clear_error();
    if (!dense || !p || !out || !bytes) return fail(VDBC_E_INVALID, "vdbc_encode: null argument");
    *out = nullptr;
    if (dims.nx == 0 || dims.ny == 0 || dims.nz == 0 || dims.nx > 0x7FFFFFFFu ||
        dims.ny > 0x7FFFFFFFu || dims.nz > 0x7FFFFFFFu)
        return fail(VDBC_E_INVALID, "vdbc_encode: dims must be in [1, 2^31)");
    if (!(p->rate > 0.0f && p->rate <= 1.0f))
        return fail(VDBC_E_INVALID, "vdbc_encode: rate must be in (0, 1]");
    if (p->metric < 1 || p->metric > 3)
        return fail(VDBC_E_INVALID, "vdbc_encode: metric must be 1, 2 or 3");
    if ((p->flags & VDBC_BG_EXPLICIT) && !std::isfinite(p->background))
        return fail(VDBC_E_INVALID, "vdbc_encode: explicit background must be finite");
    if (p->flags & ~(uint32_t)(VDBC_BG_EXPLICIT | VDBC_NO_CORNERS | VDBC_NO_PRUNE | VDBC_PARTIAL))
        return fail(VDBC_E_INVALID, "vdbc_encode: unknown flag bits 0x%x", p->flags);
    if ((p->flags & VDBC_PARTIAL) &&
        (!(p->partial_fraction > 0.0f && p->partial_fraction <= 1.0f) || std::isnan(p->partial_threshold)))
        return fail(VDBC_E_INVALID, "vdbc_encode: partial fraction must be in (0, 1] and the threshold not NaN");
    std::unique_ptr<vdbc_encoder> e(new (std::nothrow) vdbc_encoder());
    if (!e) return fail(VDBC_E_NOMEM, "vdbc_encode: no memory");
    e->dense = dense;
    e->nx = dims.nx;
    e->ny = dims.ny;
    e->nz = dims.nz;
    e->p = *p;
    e->threads = worker_count(p->threads);
    e->nbx = cdiv(e->nx, kBrick);
    e->nby = cdiv(e->ny, kBrick);
    e->nbz = cdiv(e->nz, kBrick);
    e->N = (uint64_t)e->nbx * e->nby * e->nbz;
    try {
        std::vector<float> lo(e->N), hi(e->N);
        std::vector<uint64_t> hist;
        vdbc_status s = scan_ranges_and_histogram(*e, lo, hi, hist);
        if (s) return s;
        if (p->flags & VDBC_BG_EXPLICIT) {
            e->B = p->background;
        } else {
            s = background_mode(*e, hist);
            if (s) return s;
        }
        // step 3: similarity (Eq. 1-3, double) and sort
        std::vector<double> f(e->N);
        const double B = (double)e->B;
        for (uint64_t b = 0; b < e->N; ++b) {
            double dl = std::fabs((double)lo[b] - B), dh = std::fabs((double)hi[b] - B);
            if (p->metric == 1) f[b] = dl < dh ? dl : dh;
            else if (p->metric == 3) f[b] = std::fabs(((double)lo[b] + (double)hi[b]) / 2.0 - B);
            else f[b] = dl > dh ? dl : dh;
        }
        std::vector<uint32_t> order(e->N);
        for (uint64_t b = 0; b < e->N; ++b) order[b] = (uint32_t)b;
        std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
            return f[a] > f[b] || (f[a] == f[b] && a < b);
        });
        uint64_t K = (uint64_t)std::floor((double)p->rate * (double)e->N + 0.5);
        e->K = K > e->N ? e->N : K;
        // step 4: activation (whole bricks: the first K, or with VDBC_PARTIAL
        // the first F that reach the threshold, plus any partial-region brick
        // the budget covers completely)
        uint64_t F = e->K;
        if (p->flags & VDBC_PARTIAL) {
            const double tau = (double)p->partial_threshold;
            F = 0;
            while (F < e->K && f[order[F]] >= tau) ++F;
        }
        e->brick_sel.assign(e->N, 0);
        std::vector<uint32_t> selected(order.begin(), order.begin() + F);
        e->partial.clear();
        e->brick_part.clear();
        if (F < e->K) {
            s = plan_partial(*e, order, F, selected);
            if (s) return s;
        }
        std::sort(selected.begin(), selected.end());
        for (uint32_t b : selected) e->brick_sel[b] = 1;
        uint64_t active = 0;
        for (uint32_t b : selected) active += brick_voxels(*e, b);
        for (const PartialBrick& P : e->partial) active += P.count;
        if (!(p->flags & VDBC_NO_CORNERS)) {
            const uint64_t cx[2] = {0, e->nx - 1u}, cy[2] = {0, e->ny - 1u}, cz[2] = {0, e->nz - 1u};
            const bool same = (e->nx == 1 && e->ny == 1 && e->nz == 1);
            for (int c = 0; c < (same ? 1 : 2); ++c) {
                const uint32_t b = (uint32_t)(cx[c] / kBrick) +
                                   e->nbx * ((uint32_t)(cy[c] / kBrick) + e->nby * (uint32_t)(cz[c] / kBrick));
                if (e->brick_sel[b]) continue;
                const uint32_t pi = e->partial.empty() ? kNoChild : e->brick_part[b];
                if (pi != kNoChild && partial_active(*e, e->partial[pi], cx[c], cy[c], cz[c])) continue;
                ++active;
            }
        }
        e->active = active;
        s = build_tree(*e, selected);
        if (s) return s;
        fill_header(*e);
    } catch (const std::bad_alloc&) {
        return fail(VDBC_E_NOMEM, "vdbc_encode: out of host memory");
    }
    *bytes = e->h.total_bytes;
    if (stats) {
        stats->background = e->B;
        stats->n_bricks = e->N;
        stats->k_bricks = e->K;
        stats->n_leaf = e->n_leaf;
        stats->n_lower = e->n_lower;
        stats->n_upper = e->n_upper;
        stats->n_lower_tiles = e->n_ltile;
        stats->n_upper_tiles = e->n_utile;
        stats->active_voxels = e->active;
        stats->bytes = e->h.total_bytes;
        stats->achieved_rate = (double)e->active / ((double)e->nx * e->ny * e->nz);
    }
    *out = e.release();
    return VDBC_OK;
}

extern "C" void vdbc_encode_abort(vdbc_encoder* h) { delete h; }

extern "C" vdbc_status vdbc_encode_finish(vdbc_encoder* hnd, void* out_v, uint64_t capacity)
{
    clear_error();
    std::unique_ptr<vdbc_encoder> e(hnd);
    if (!e) return fail(VDBC_E_INVALID, "vdbc_encode_finish: null handle");
    if (!out_v) return fail(VDBC_E_INVALID, "vdbc_encode_finish: null output");
    const Header& h = e->h;
    if (capacity < h.total_bytes)
        return fail(VDBC_E_BUFFER_TOO_SMALL, "vdbc_encode_finish: capacity %llu < %llu bytes",
                    (unsigned long long)capacity, (unsigned long long)h.total_bytes);
    uint8_t* o = static_cast<uint8_t*>(out_v);
    try {
        write_header(h, o);
        // everything before the leaf values is small: zero it, then fill
        std::memset(o + kHeaderBytes, 0, h.off_leaf_values - kHeaderBytes);
        std::memset(o + h.off_leaf_values + 2048 * e->n_leaf, 0,
                    h.total_bytes - (h.off_leaf_values + 2048 * e->n_leaf));
        uint64_t rn = (uint64_t)e->rnx * e->rny * e->rnz;
        for (uint64_t r = 0; r < rn; ++r) put<uint32_t>(o, h.off_root + 4 * r, kNoChild);
        for (uint64_t u = 0; u < e->n_upper; ++u)
            put<uint32_t>(o, h.off_root + 4 * e->upper_root[u], (uint32_t)u);
        Word* uw = reinterpret_cast<Word*>(o + h.off_upper);
        Word* lw = reinterpret_cast<Word*>(o + h.off_lower);
        float* ut = reinterpret_cast<float*>(o + h.off_upper_tiles);
        float* lt = reinterpret_cast<float*>(o + h.off_lower_tiles);
        // leaf numbering
        std::vector<uint32_t> leaf_slot(e->leaves.size(), kNoChild);
        uint32_t lower_i = 0, leaf_i = 0, utile_i = 0, ltile_i = 0;
        size_t li = 0;
        for (uint64_t u = 0; u < e->n_upper; ++u) {
            Word* node = uw + (uint64_t)u * kUpperWords;
            uint64_t r = e->upper_root[u];
            for (uint32_t w = 0; w < kUpperWords; ++w) {
                node[w].child_index = lower_i;
                node[w].tile_index = utile_i;
                while (li < e->lowers.size() && (e->lowers[li].key >> 15) == r &&
                       (uint32_t)((e->lowers[li].key & 0x7FFF) >> 6) == w) {
                    const LowerRec& L = e->lowers[li];
                    uint32_t n1 = (uint32_t)(L.key & 0x7FFF);
                    uint64_t bit = uint64_t(1) << (n1 & 63);
                    if (L.is_tile) {
                        node[w].tile |= bit;
                        float v;
                        std::memcpy(&v, &L.tile_bits, 4);
                        ut[utile_i++] = v;
                    } else {
                        node[w].child |= bit;
                        Word* lnode = lw + (uint64_t)lower_i * kLowerWords;
                        ++lower_i;
                        size_t lf = L.first;
                        for (uint32_t w2 = 0; w2 < kLowerWords; ++w2) {
                            lnode[w2].child_index = leaf_i;
                            lnode[w2].tile_index = ltile_i;
                            while (lf < L.first + L.count &&
                                   (uint32_t)((e->leaves[lf].key & 0xFFF) >> 6) == w2) {
                                const LeafRec& F = e->leaves[lf];
                                uint64_t b2 = uint64_t(1) << ((F.key & 0xFFF) & 63);
                                if (F.is_tile) {
                                    lnode[w2].tile |= b2;
                                    float v;
                                    std::memcpy(&v, &F.tile_bits, 4);
                                    lt[ltile_i++] = v;
                                } else {
                                    lnode[w2].child |= b2;
                                    leaf_slot[lf] = leaf_i++;
                                }
                                ++lf;
                            }
                        }
                    }
                    ++li;
                }
            }
        }
        // leaf masks and values (the bulk of the bytes), in parallel
        uint64_t* masks = reinterpret_cast<uint64_t*>(o + h.off_leaf_masks);
        float* vals = reinterpret_cast<float*>(o + h.off_leaf_values);
        const float B = e->B;
        parallel_for(e->leaves.size(), e->threads, [&](uint64_t i, unsigned) {
            uint32_t slot = leaf_slot[i];
            if (slot == kNoChild) return;
            const LeafRec& F = e->leaves[i];
            uint64_t* m = masks + 8ull * slot;
            float* v = vals + 512ull * slot;
            for (int q = 0; q < 8; ++q) m[q] = 0;
            for (uint32_t k = 0; k < 8; ++k)
                for (uint32_t j = 0; j < 8; ++j) {
                    uint64_t z = 8ull * F.lz + k, y = 8ull * F.ly + j;
                    for (uint32_t i3 = 0; i3 < 8; ++i3) {
                        uint64_t x = 8ull * F.lx + i3;
                        uint32_t n3 = i3 + 8 * (j + 8 * k);
                        float val = B;
                        if (x < e->nx && y < e->ny && z < e->nz) {
                            bool act = leaf_voxel_active(*e, F, x, y, z);
                            if (act) {
                                val = e->dense[voxel_index(*e, x, y, z)];
                                m[n3 >> 6] |= uint64_t(1) << (n3 & 63);
                            }
                        }
                        v[n3] = val;
                    }
                }
        });
    } catch (const std::bad_alloc&) {
        return fail(VDBC_E_NOMEM, "vdbc_encode_finish: out of host memory");
    }
    return VDBC_OK;
}

extern "C" vdbc_status vdbc_encode(const float* dense, vdbc_dims dims,
                                   const vdbc_encode_params* p, void* out, uint64_t capacity,
                                   uint64_t* bytes, vdbc_encode_stats* stats)
{
    vdbc_encoder* h = nullptr;
    uint64_t need = 0;
    vdbc_status s = vdbc_encode_begin(dense, dims, p, &h, &need, stats);
    if (s) return s;
    if (bytes) *bytes = need;
    if (!out || capacity < need) {
        vdbc_encode_abort(h);
        return fail(VDBC_E_BUFFER_TOO_SMALL, "vdbc_encode: need %llu bytes",
                    (unsigned long long)need);
    }
    return vdbc_encode_finish(h, out, capacity);
}
