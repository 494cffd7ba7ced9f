/* Oracle encoder: Alg. 1 "Compress" (Section 3.1) and the tree construction
 * and linearisation of Section 3.2, written as plain loops over voxels.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Readings where the paper is silent or garbled (each is also listed in the
 * design notes):
 *  - tree levels: 8^3 leaves, 16^3-child lower nodes, 32^3-child upper nodes
 *    (the Tree4<float,5,4,3> of Section 3.2.1; the level sizes printed next to
 *    Alg. 1 are inverted);
 *  - background: exact mode of the float values, -0 counted as +0, ties to the
 *    numerically smallest value (Alg. 1 histogram + argmax);
 *  - bricks: ceil(dims/32) with partial edge bricks, ranges over in-volume
 *    voxels;
 *  - sort: similarity descending = most dissimilar from B first, ties by the
 *    x-fastest brick index ascending; the first K bricks are activated with
 *    K = min(N, floor(q*N + 0.5));
 *  - corners: voxels (0,0,0) and (nx-1,ny-1,nz-1) are always active
 *    (Section 3.2.1) unless REF_NO_CORNERS;
 *  - partial-brick activation (REF_PARTIAL; the variant Section 3.2.1 leaves
 *    as future work, no rule given there): with fraction p and similarity
 *    threshold tau, the first F = #{r < K : f_r >= tau} ranked bricks are
 *    activated whole and the voxels of the bricks ranked K..F-1 under plain
 *    Alg. 1, R = sum of their in-volume voxel counts, are spent instead along
 *    the bricks ranked F, F+1, ...: first ceil(p * v_r) voxels of each brick
 *    (v_r = its in-volume voxels), then, once every brick had its share, the
 *    rest of each brick in rank order; inside a brick voxels go by |value - B|
 *    descending (double), ties by linear voxel index ascending.  The first R
 *    voxels of that sequence are activated.  p = 1 or tau below every
 *    similarity gives Alg. 1 itself;
 *  - inactive voxels inside a leaf store B; prune at tolerance 0: a leaf whose
 *    512 voxels are all active and bitwise equal becomes a lower-node tile, a
 *    lower node whose 4096 slots are all such tiles of one value becomes an
 *    upper-node tile; upper nodes are never pruned.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define BRICK 32u

static uint32_t fbits(float v)
{
    uint32_t b;
    memcpy(&b, &v, 4);
    return b;
}

static int cmp_float(const void* a, const void* b)
{
    float x = *(const float*)a, y = *(const float*)b;
    return (x < y) ? -1 : (x > y) ? 1 : 0;
}

float ref_background(const float* dense, uint64_t n)
{
    float* v = (float*)malloc(n * sizeof(float));
    if (!v) return NAN;
    for (uint64_t i = 0; i < n; ++i) v[i] = (dense[i] == 0.0f) ? 0.0f : dense[i];
    qsort(v, n, sizeof(float), cmp_float);
    float best = v[0];
    uint64_t best_count = 0;
    uint64_t i = 0;
    while (i < n) {
        uint64_t j = i;
        while (j < n && v[j] == v[i]) ++j;
        if (j - i > best_count) { /* strictly greater: ties keep the smaller value */
            best_count = j - i;
            best = v[i];
        }
        i = j;
    }
    free(v);
    return best;
}

static uint32_t ceil_div(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

void ref_brick_ranges(const float* dense, uint32_t nx, uint32_t ny, uint32_t nz,
                      float* lo, float* hi)
{
    uint32_t nbx = ceil_div(nx, BRICK), nby = ceil_div(ny, BRICK), nbz = ceil_div(nz, BRICK);
    for (uint32_t bz = 0; bz < nbz; ++bz)
        for (uint32_t by = 0; by < nby; ++by)
            for (uint32_t bx = 0; bx < nbx; ++bx) {
                uint64_t b = bx + (uint64_t)nbx * (by + (uint64_t)nby * bz);
                float l = INFINITY, h = -INFINITY;
                for (uint32_t z = bz * BRICK; z < nz && z < (bz + 1) * BRICK; ++z)
                    for (uint32_t y = by * BRICK; y < ny && y < (by + 1) * BRICK; ++y)
                        for (uint32_t x = bx * BRICK; x < nx && x < (bx + 1) * BRICK; ++x) {
                            float v = dense[x + (uint64_t)nx * (y + (uint64_t)ny * z)];
                            if (v < l) l = v;
                            if (v > h) h = v;
                        }
                lo[b] = l;
                hi[b] = h;
            }
}

/* Eq. (1) closest, (2) farthest, (3) median point-in-range distance to B. */
double ref_similarity(uint32_t metric, float lo, float hi, float B)
{
    double dl = fabs((double)lo - (double)B);
    double dh = fabs((double)hi - (double)B);
    if (metric == 1) return dl < dh ? dl : dh;
    if (metric == 3) return fabs(((double)lo + (double)hi) / 2.0 - (double)B);
    return dl > dh ? dl : dh;
}

typedef struct {
    double f;
    uint32_t idx;
} brick_key;

static int cmp_brick(const void* a, const void* b)
{
    const brick_key* x = (const brick_key*)a;
    const brick_key* y = (const brick_key*)b;
    if (x->f > y->f) return -1;
    if (x->f < y->f) return 1;
    return (x->idx < y->idx) ? -1 : (x->idx > y->idx) ? 1 : 0;
}

static int check_input(const float* dense, uint32_t nx, uint32_t ny, uint32_t nz,
                       float rate, uint32_t metric)
{
    if (!dense || nx == 0 || ny == 0 || nz == 0) return REF_E_INVALID;
    if (!(rate > 0.0f && rate <= 1.0f)) return REF_E_INVALID;
    if (metric < 1 || metric > 3) return REF_E_INVALID;
    uint64_t n = (uint64_t)nx * ny * nz;
    for (uint64_t i = 0; i < n; ++i)
        if (!isfinite(dense[i])) return REF_E_INVALID;
    return REF_OK;
}

int ref_brick_order(const float* dense, uint32_t nx, uint32_t ny, uint32_t nz,
                    float rate, uint32_t metric, float B, uint32_t* order,
                    uint64_t* k_out)
{
    uint32_t nbx = ceil_div(nx, BRICK), nby = ceil_div(ny, BRICK), nbz = ceil_div(nz, BRICK);
    uint64_t N = (uint64_t)nbx * nby * nbz;
    float* lo = (float*)malloc(N * sizeof(float));
    float* hi = (float*)malloc(N * sizeof(float));
    brick_key* keys = (brick_key*)malloc(N * sizeof(brick_key));
    if (!lo || !hi || !keys) {
        free(lo);
        free(hi);
        free(keys);
        return REF_E_NOMEM;
    }
    ref_brick_ranges(dense, nx, ny, nz, lo, hi);
    for (uint64_t b = 0; b < N; ++b) {
        keys[b].f = ref_similarity(metric, lo[b], hi[b], B);
        keys[b].idx = (uint32_t)b;
    }
    qsort(keys, N, sizeof(brick_key), cmp_brick);
    for (uint64_t b = 0; b < N; ++b) order[b] = keys[b].idx;
    uint64_t K = (uint64_t)floor((double)rate * (double)N + 0.5);
    if (K > N) K = N;
    *k_out = K;
    free(lo);
    free(hi);
    free(keys);
    return REF_OK;
}

typedef struct {
    double d;       /* |value - B| */
    uint64_t idx;   /* linear voxel index */
} voxel_key;

static int cmp_voxel(const void* a, const void* b)
{
    const voxel_key* x = (const voxel_key*)a;
    const voxel_key* y = (const voxel_key*)b;
    if (x->d > y->d) return -1;
    if (x->d < y->d) return 1;
    return (x->idx < y->idx) ? -1 : (x->idx > y->idx) ? 1 : 0;
}

static uint64_t brick_voxels(uint32_t b, uint32_t nbx, uint32_t nby, uint32_t nx, uint32_t ny,
                             uint32_t nz)
{
    uint32_t bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    uint64_t ex = nx - bx * BRICK < BRICK ? nx - bx * BRICK : BRICK;
    uint64_t ey = ny - by * BRICK < BRICK ? ny - by * BRICK : BRICK;
    uint64_t ez = nz - bz * BRICK < BRICK ? nz - bz * BRICK : BRICK;
    return ex * ey * ez;
}

/* The in-volume voxels of brick b ordered by |value - B| descending, ties by
 * linear index ascending (the voxel order inside a partially active brick). */
static voxel_key* brick_voxel_order(const float* dense, uint32_t b, uint32_t nbx, uint32_t nby,
                                    uint32_t nx, uint32_t ny, uint32_t nz, float B, uint64_t* count)
{
    uint32_t bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    uint64_t v = brick_voxels(b, nbx, nby, nx, ny, nz), c = 0;
    voxel_key* keys = (voxel_key*)malloc(v * sizeof(voxel_key));
    if (!keys) return NULL;
    for (uint32_t z = bz * BRICK; z < nz && z < (bz + 1) * BRICK; ++z)
        for (uint32_t y = by * BRICK; y < ny && y < (by + 1) * BRICK; ++y)
            for (uint32_t x = bx * BRICK; x < nx && x < (bx + 1) * BRICK; ++x) {
                uint64_t i = x + (uint64_t)nx * (y + (uint64_t)ny * z);
                keys[c].d = fabs((double)dense[i] - (double)B);
                keys[c].idx = i;
                ++c;
            }
    qsort(keys, c, sizeof(voxel_key), cmp_voxel);
    *count = c;
    return keys;
}

/* Activation mask: all in-volume voxels of the first K bricks + corners, or
 * with REF_PARTIAL the partial-brick rule described at the top of the file. */
static int activation(const float* dense, uint32_t nx, uint32_t ny, uint32_t nz,
                      float rate, uint32_t metric, uint32_t flags, float bg,
                      float pfrac, float ptau,
                      uint8_t** active_out, float* B_out, uint64_t* N_out,
                      uint64_t* K_out)
{
    int rc = check_input(dense, nx, ny, nz, rate, metric);
    if (rc) return rc;
    if ((flags & REF_PARTIAL) && (!(pfrac > 0.0f && pfrac <= 1.0f) || isnan(ptau)))
        return REF_E_INVALID;
    uint64_t n = (uint64_t)nx * ny * nz;
    float B;
    if (flags & REF_BG_EXPLICIT) {
        if (!isfinite(bg)) return REF_E_INVALID;
        B = bg;
    } else {
        B = ref_background(dense, n);
    }
    uint32_t nbx = ceil_div(nx, BRICK), nby = ceil_div(ny, BRICK), nbz = ceil_div(nz, BRICK);
    uint64_t N = (uint64_t)nbx * nby * nbz;
    uint32_t* order = (uint32_t*)malloc(N * sizeof(uint32_t));
    uint8_t* active = (uint8_t*)calloc(n, 1);
    if (!order || !active) {
        free(order);
        free(active);
        return REF_E_NOMEM;
    }
    uint64_t K = 0;
    rc = ref_brick_order(dense, nx, ny, nz, rate, metric, B, order, &K);
    if (rc) {
        free(order);
        free(active);
        return rc;
    }
    /* bricks activated whole: the first K, or with REF_PARTIAL the first F */
    uint64_t F = K;
    if (flags & REF_PARTIAL) {
        /* similarities of the ranked bricks, recomputed as in ref_brick_order */
        float* lo = (float*)malloc(N * sizeof(float));
        float* hi = (float*)malloc(N * sizeof(float));
        if (!lo || !hi) {
            free(lo);
            free(hi);
            free(order);
            free(active);
            return REF_E_NOMEM;
        }
        ref_brick_ranges(dense, nx, ny, nz, lo, hi);
        F = 0;
        while (F < K && ref_similarity(metric, lo[order[F]], hi[order[F]], B) >= (double)ptau) ++F;
        free(lo);
        free(hi);
    }
    for (uint64_t s = 0; s < F; ++s) {
        uint32_t b = order[s];
        uint32_t bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
        for (uint32_t z = bz * BRICK; z < nz && z < (bz + 1) * BRICK; ++z)
            for (uint32_t y = by * BRICK; y < ny && y < (by + 1) * BRICK; ++y)
                for (uint32_t x = bx * BRICK; x < nx && x < (bx + 1) * BRICK; ++x)
                    active[x + (uint64_t)nx * (y + (uint64_t)ny * z)] = 1;
    }
    if (F < K) {
        /* the budget: the voxels of the bricks ranked F..K-1 */
        uint64_t R = 0;
        for (uint64_t s = F; s < K; ++s) R += brick_voxels(order[s], nbx, nby, nx, ny, nz);
        /* first sweep: ceil(p v) voxels of each brick from rank F on;
         * second sweep: the rest of each brick, in the same rank order */
        for (int sweep = 0; sweep < 2 && R > 0; ++sweep)
            for (uint64_t s = F; s < N && R > 0; ++s) {
                uint64_t cnt = 0;
                voxel_key* keys = brick_voxel_order(dense, order[s], nbx, nby, nx, ny, nz, B, &cnt);
                if (!keys) {
                    free(order);
                    free(active);
                    return REF_E_NOMEM;
                }
                uint64_t share = (uint64_t)ceil((double)pfrac * (double)cnt);
                if (share > cnt) share = cnt;
                uint64_t a = sweep == 0 ? 0 : share, e = sweep == 0 ? share : cnt;
                for (uint64_t j = a; j < e && R > 0; ++j, --R) active[keys[j].idx] = 1;
                free(keys);
            }
    }
    if (!(flags & REF_NO_CORNERS)) {
        active[0] = 1;
        active[n - 1] = 1;
    }
    free(order);
    *active_out = active;
    *B_out = B;
    *N_out = N;
    *K_out = K;
    return REF_OK;
}

int ref_reconstruct_partial(const float* dense, uint32_t nx, uint32_t ny, uint32_t nz,
                            float rate, uint32_t metric, uint32_t flags, float bg, float pfrac,
                            float ptau, float* R)
{
    uint8_t* active = NULL;
    float B;
    uint64_t N, K;
    int rc = activation(dense, nx, ny, nz, rate, metric, flags, bg, pfrac, ptau, &active, &B, &N, &K);
    if (rc) return rc;
    uint64_t n = (uint64_t)nx * ny * nz;
    for (uint64_t i = 0; i < n; ++i) R[i] = active[i] ? dense[i] : B;
    free(active);
    return REF_OK;
}

int ref_reconstruct(const float* dense, uint32_t nx, uint32_t ny, uint32_t nz,
                    float rate, uint32_t metric, uint32_t flags, float bg, float* R)
{
    if (flags & REF_PARTIAL) return REF_E_INVALID;
    return ref_reconstruct_partial(dense, nx, ny, nz, rate, metric, flags, bg, 1.0f, 0.0f, R);
}

int ref_active_mask(const float* dense, uint32_t nx, uint32_t ny, uint32_t nz, float rate,
                    uint32_t metric, uint32_t flags, float bg, float pfrac, float ptau,
                    uint8_t* mask)
{
    uint8_t* active = NULL;
    float B;
    uint64_t N, K;
    int rc = activation(dense, nx, ny, nz, rate, metric, flags, bg, pfrac, ptau, &active, &B, &N, &K);
    if (rc) return rc;
    memcpy(mask, active, (uint64_t)nx * ny * nz);
    free(active);
    return REF_OK;
}

/* ---------------- tree construction and linearisation ---------------- */

enum { S_EMPTY = 0, S_NODE = 1, S_TILE = 2 };

static uint64_t align256(uint64_t x) { return (x + 255u) & ~(uint64_t)255u; }

static void put32(uint8_t* p, uint32_t v) { memcpy(p, &v, 4); }
static void put64(uint8_t* p, uint64_t v) { memcpy(p, &v, 8); }
static void putf(uint8_t* p, float v) { memcpy(p, &v, 4); }

int ref_encode(const float* dense, uint32_t nx, uint32_t ny, uint32_t nz,
               float rate, uint32_t metric, uint32_t flags, float bg,
               uint8_t** out, uint64_t* bytes, ref_stats* st)
{
    if (flags & REF_PARTIAL) return REF_E_INVALID;
    return ref_encode_partial(dense, nx, ny, nz, rate, metric, flags, bg, 1.0f, 0.0f, out, bytes, st);
}

int ref_encode_partial(const float* dense, uint32_t nx, uint32_t ny, uint32_t nz,
                       float rate, uint32_t metric, uint32_t flags, float bg, float pfrac,
                       float ptau, uint8_t** out, uint64_t* bytes, ref_stats* st)
{
    uint8_t* active = NULL;
    float B;
    uint64_t N, K;
    int rc = activation(dense, nx, ny, nz, rate, metric, flags, bg, pfrac, ptau, &active, &B, &N, &K);
    if (rc) return rc;
    const int prune = !(flags & REF_NO_PRUNE);
    uint64_t n = (uint64_t)nx * ny * nz;
    uint64_t n_active = 0;
    for (uint64_t i = 0; i < n; ++i) n_active += active[i];

    /* Level grids: leaves cover 8^3 voxels, lower nodes 128^3, uppers 4096^3. */
    uint32_t lx = ceil_div(nx, 8), ly = ceil_div(ny, 8), lz = ceil_div(nz, 8);
    uint32_t Lx = ceil_div(nx, 128), Ly = ceil_div(ny, 128), Lz = ceil_div(nz, 128);
    uint32_t Ux = ceil_div(nx, 4096), Uy = ceil_div(ny, 4096), Uz = ceil_div(nz, 4096);
    uint64_t n_leafgrid = (uint64_t)lx * ly * lz;
    uint64_t n_lowergrid = (uint64_t)Lx * Ly * Lz;
    uint64_t n_uppergrid = (uint64_t)Ux * Uy * Uz;

    uint8_t* leaf_state = (uint8_t*)calloc(n_leafgrid, 1);
    uint32_t* leaf_tile = (uint32_t*)calloc(n_leafgrid, 4);       /* tile value bits */
    uint8_t* lower_state = (uint8_t*)calloc(n_lowergrid, 1);
    uint32_t* lower_tile = (uint32_t*)calloc(n_lowergrid, 4);
    uint8_t* upper_state = (uint8_t*)calloc(n_uppergrid, 1);
    if (!leaf_state || !leaf_tile || !lower_state || !lower_tile || !upper_state) {
        rc = REF_E_NOMEM;
        goto done;
    }

    /* Leaves exist wherever a voxel is active; prune uniform full leaves. */
    for (uint32_t z = 0; z < lz; ++z)
        for (uint32_t y = 0; y < ly; ++y)
            for (uint32_t x = 0; x < lx; ++x) {
                uint64_t li = x + (uint64_t)lx * (y + (uint64_t)ly * z);
                uint32_t count = 0, first = 0, uniform = 1;
                for (uint32_t k = 0; k < 8; ++k)
                    for (uint32_t j = 0; j < 8; ++j)
                        for (uint32_t i = 0; i < 8; ++i) {
                            uint64_t X = 8u * x + i, Y = 8u * y + j, Z = 8u * z + k;
                            if (X >= nx || Y >= ny || Z >= nz) continue;
                            uint64_t v = X + nx * (Y + ny * Z);
                            if (!active[v]) continue;
                            uint32_t b = fbits(dense[v]);
                            if (count == 0) first = b;
                            else if (b != first) uniform = 0;
                            ++count;
                        }
                if (count == 0) continue;
                if (prune && count == 512 && uniform) {
                    leaf_state[li] = S_TILE;
                    leaf_tile[li] = first;
                } else {
                    leaf_state[li] = S_NODE;
                }
            }

    /* Lower nodes exist wherever a slot holds a leaf or a tile. */
    for (uint32_t z = 0; z < Lz; ++z)
        for (uint32_t y = 0; y < Ly; ++y)
            for (uint32_t x = 0; x < Lx; ++x) {
                uint64_t Li = x + (uint64_t)Lx * (y + (uint64_t)Ly * z);
                uint32_t any = 0, tiles = 0, first = 0, uniform = 1;
                for (uint32_t k = 0; k < 16; ++k)
                    for (uint32_t j = 0; j < 16; ++j)
                        for (uint32_t i = 0; i < 16; ++i) {
                            uint64_t X = 16u * x + i, Y = 16u * y + j, Z = 16u * z + k;
                            if (X >= lx || Y >= ly || Z >= lz) continue;
                            uint64_t li = X + lx * (Y + ly * Z);
                            if (leaf_state[li] == S_EMPTY) continue;
                            any = 1;
                            if (leaf_state[li] == S_TILE) {
                                if (tiles == 0) first = leaf_tile[li];
                                else if (leaf_tile[li] != first) uniform = 0;
                                ++tiles;
                            }
                        }
                if (!any) continue;
                if (prune && tiles == 4096 && uniform) {
                    lower_state[Li] = S_TILE;
                    lower_tile[Li] = first;
                } else {
                    lower_state[Li] = S_NODE;
                }
            }

    for (uint32_t z = 0; z < Uz; ++z)
        for (uint32_t y = 0; y < Uy; ++y)
            for (uint32_t x = 0; x < Ux; ++x) {
                uint64_t Ui = x + (uint64_t)Ux * (y + (uint64_t)Uy * z);
                for (uint32_t k = 0; k < 32 && !upper_state[Ui]; ++k)
                    for (uint32_t j = 0; j < 32 && !upper_state[Ui]; ++j)
                        for (uint32_t i = 0; i < 32; ++i) {
                            uint64_t X = 32u * x + i, Y = 32u * y + j, Z = 32u * z + k;
                            if (X >= Lx || Y >= Ly || Z >= Lz) continue;
                            if (lower_state[X + Lx * (Y + Ly * Z)] != S_EMPTY) {
                                upper_state[Ui] = S_NODE;
                                break;
                            }
                        }
            }

    /* Canonical numbering: uppers by root slot, lowers by (upper, slot),
     * leaves by (lower, slot), tiles likewise. */
    uint64_t n_upper = 0, n_lower = 0, n_leaf = 0, n_utile = 0, n_ltile = 0;
    for (uint64_t Ui = 0; Ui < n_uppergrid; ++Ui) n_upper += (upper_state[Ui] == S_NODE);
    for (uint64_t Li = 0; Li < n_lowergrid; ++Li) {
        n_lower += (lower_state[Li] == S_NODE);
        n_utile += (lower_state[Li] == S_TILE);
    }
    for (uint64_t li = 0; li < n_leafgrid; ++li) {
        /* leaves and tiles below a pruned lower node are dropped */
        uint32_t x = (uint32_t)(li % lx), y = (uint32_t)((li / lx) % ly), z = (uint32_t)(li / ((uint64_t)lx * ly));
        uint64_t Li = (x / 16) + (uint64_t)Lx * ((y / 16) + (uint64_t)Ly * (z / 16));
        if (lower_state[Li] != S_NODE) continue;
        n_leaf += (leaf_state[li] == S_NODE);
        n_ltile += (leaf_state[li] == S_TILE);
    }

    uint64_t off_root = 256;
    uint64_t off_upper = align256(off_root + 4 * n_uppergrid);
    uint64_t off_lower = align256(off_upper + n_upper * 512u * 32u);
    uint64_t off_utile = align256(off_lower + n_lower * 64u * 32u);
    uint64_t off_ltile = align256(off_utile + 4 * n_utile);
    uint64_t off_lmask = align256(off_ltile + 4 * n_ltile);
    uint64_t off_lval = align256(off_lmask + 64 * n_leaf);
    uint64_t total = align256(off_lval + 2048 * n_leaf);

    uint8_t* buf = (uint8_t*)calloc(total, 1);
    if (!buf) {
        rc = REF_E_NOMEM;
        goto done;
    }

    memcpy(buf, "VDBC", 4);
    put32(buf + 4, 1);
    put32(buf + 8, nx);
    put32(buf + 12, ny);
    put32(buf + 16, nz);
    putf(buf + 20, B);
    putf(buf + 24, rate);
    put32(buf + 28, metric);
    put32(buf + 32, flags);
    put32(buf + 36, 0);
    put64(buf + 40, N);
    put64(buf + 48, K);
    put64(buf + 56, n_active);
    put32(buf + 64, (uint32_t)n_upper);
    put32(buf + 68, (uint32_t)n_lower);
    put32(buf + 72, (uint32_t)n_leaf);
    put32(buf + 76, (uint32_t)n_utile);
    put32(buf + 80, (uint32_t)n_ltile);
    put32(buf + 84, Ux);
    put32(buf + 88, Uy);
    put32(buf + 92, Uz);
    put64(buf + 96, off_root);
    put64(buf + 104, off_upper);
    put64(buf + 112, off_lower);
    put64(buf + 120, off_utile);
    put64(buf + 128, off_ltile);
    put64(buf + 136, off_lmask);
    put64(buf + 144, off_lval);
    put64(buf + 152, total);
    if (flags & REF_PARTIAL) {
        putf(buf + 160, pfrac);
        putf(buf + 164, ptau);
    }

    uint32_t up_i = 0, lo_i = 0, leaf_i = 0, ut_i = 0, lt_i = 0;
    for (uint32_t uz = 0; uz < Uz; ++uz)
        for (uint32_t uy = 0; uy < Uy; ++uy)
            for (uint32_t ux = 0; ux < Ux; ++ux) {
                uint64_t Ui = ux + (uint64_t)Ux * (uy + (uint64_t)Uy * uz);
                if (upper_state[Ui] != S_NODE) {
                    put32(buf + off_root + 4 * Ui, 0xFFFFFFFFu);
                    continue;
                }
                put32(buf + off_root + 4 * Ui, up_i);
                uint8_t* unode = buf + off_upper + (uint64_t)up_i * 512u * 32u;
                ++up_i;
                for (uint32_t n1 = 0; n1 < 32768; ++n1) {
                    uint8_t* rec = unode + (n1 / 64) * 32u;
                    if (n1 % 64 == 0) {
                        put32(rec + 8, lo_i);
                        put32(rec + 12, ut_i);
                    }
                    uint32_t X = 32u * ux + (n1 & 31), Y = 32u * uy + ((n1 >> 5) & 31),
                             Z = 32u * uz + (n1 >> 10);
                    if (X >= Lx || Y >= Ly || Z >= Lz) continue;
                    uint64_t Li = X + (uint64_t)Lx * (Y + (uint64_t)Ly * Z);
                    uint64_t bit = (uint64_t)1 << (n1 % 64);
                    if (lower_state[Li] == S_TILE) {
                        uint64_t m;
                        memcpy(&m, rec + 16, 8);
                        put64(rec + 16, m | bit);
                        put32(buf + off_utile + 4u * ut_i, lower_tile[Li]);
                        ++ut_i;
                        continue;
                    }
                    if (lower_state[Li] != S_NODE) continue;
                    uint64_t m;
                    memcpy(&m, rec, 8);
                    put64(rec, m | bit);
                    uint8_t* lnode = buf + off_lower + (uint64_t)lo_i * 64u * 32u;
                    ++lo_i;
                    for (uint32_t n2 = 0; n2 < 4096; ++n2) {
                        uint8_t* r2 = lnode + (n2 / 64) * 32u;
                        if (n2 % 64 == 0) {
                            put32(r2 + 8, leaf_i);
                            put32(r2 + 12, lt_i);
                        }
                        uint32_t x = 16u * X + (n2 & 15), y = 16u * Y + ((n2 >> 4) & 15),
                                 z = 16u * Z + (n2 >> 8);
                        if (x >= lx || y >= ly || z >= lz) continue;
                        uint64_t li = x + (uint64_t)lx * (y + (uint64_t)ly * z);
                        uint64_t b2 = (uint64_t)1 << (n2 % 64);
                        if (leaf_state[li] == S_TILE) {
                            uint64_t m2;
                            memcpy(&m2, r2 + 16, 8);
                            put64(r2 + 16, m2 | b2);
                            put32(buf + off_ltile + 4u * lt_i, leaf_tile[li]);
                            ++lt_i;
                            continue;
                        }
                        if (leaf_state[li] != S_NODE) continue;
                        uint64_t m2;
                        memcpy(&m2, r2, 8);
                        put64(r2, m2 | b2);
                        uint8_t* mask = buf + off_lmask + 64u * (uint64_t)leaf_i;
                        uint8_t* vals = buf + off_lval + 2048u * (uint64_t)leaf_i;
                        ++leaf_i;
                        for (uint32_t n3 = 0; n3 < 512; ++n3) {
                            uint64_t vx = 8u * (uint64_t)x + (n3 & 7), vy = 8u * (uint64_t)y + ((n3 >> 3) & 7),
                                     vz = 8u * (uint64_t)z + (n3 >> 6);
                            float val = B;
                            if (vx < nx && vy < ny && vz < nz) {
                                uint64_t v = vx + nx * (vy + ny * vz);
                                if (active[v]) {
                                    val = dense[v];
                                    uint64_t mw;
                                    memcpy(&mw, mask + 8 * (n3 / 64), 8);
                                    put64(mask + 8 * (n3 / 64), mw | ((uint64_t)1 << (n3 % 64)));
                                }
                            }
                            putf(vals + 4u * n3, val);
                        }
                    }
                }
            }

    *out = buf;
    *bytes = total;
    if (st) {
        st->background = B;
        st->n_bricks = N;
        st->k_bricks = K;
        st->n_leaf = n_leaf;
        st->n_lower = n_lower;
        st->n_upper = n_upper;
        st->n_lower_tiles = n_ltile;
        st->n_upper_tiles = n_utile;
        st->active_voxels = n_active;
        st->bytes = total;
        st->achieved_rate = (double)n_active / (double)n;
    }
    rc = REF_OK;
done:
    free(active);
    free(leaf_state);
    free(leaf_tile);
    free(lower_state);
    free(lower_tile);
    free(upper_state);
    return rc;
}

void ref_free(void* p) { free(p); }
