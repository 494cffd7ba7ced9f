// HIP kernels for gfx950 and their C-ABI launchers: majorant macrocells,
// emission-absorption and iso-surface marching, and the delta-tracking path
// tracer (Section 4), each for the compressed VDB and for the dense float32
// baseline through the same templated code, plus batched rendering.
#include <mutex>

#include "kcommon.h"
#include "pt.h"

namespace vdbc {

// Clears the workspace's counters: sample and cell counts, PT tile queue,
// path segment count.
__global__ void zero_u64(unsigned long long* p)
{
    if (threadIdx.x < 4 && blockIdx.x == 0) p[threadIdx.x] = 0ull;
}

// ---------------------------------------------------------------- majorant

// One workgroup per macrocell: min and max of the values of the (C+2)^3
// dilated footprint, reduced across the workgroup.  A dense array is read
// voxel by voxel (thread -> z-column).  A VDB is read leaf region by leaf
// region (thread -> 8^3 block of the footprint): a tile or an empty region
// gives its one value without touching its voxels, a stored leaf its values
// inside the footprint, so the empty space that makes up most of a
// compressed volume costs one lookup per 512 voxels.  Both give the min and
// max of the same values (the reconstruction, B outside), so the grids are
// identical.
// Leaf blocks a macrocell footprint can touch: (C + 2) / 8 + 2 per axis at
// the largest macrocell, 64.
constexpr int kMajorantQueue = 11 * 11 * 11;

// The majorant of macrocell `cell` of a gx x gy x .. grid, by the whole
// workgroup; thread 0 writes it.
template <class Acc>
__device__ void majorant_cell(Acc& acc, const MediumK& m, int C, int gx, int gy, uint32_t cell,
                              float* __restrict__ out)
{
    const int cx = (int)(cell % (uint32_t)gx), cy = (int)((cell / (uint32_t)gx) % (uint32_t)gy),
              cz = (int)(cell / ((uint32_t)gx * (uint32_t)gy));
    const int E = C + 2, x0 = C * cx - 1, y0 = C * cy - 1, z0 = C * cz - 1;
    float vmin = INFINITY, vmax = -INFINITY;
    if constexpr (Acc::kTree) {
        // leaf blocks [bx0, bx0 + nbx) x ... covering the footprint (floor
        // division; at most 11^3 for a macrocell of 64).  First every thread
        // resolves its blocks: a constant region enters the min and max at
        // once, a stored leaf is queued in LDS.  Then each wave reads the
        // queued leaves whole, 8 voxels per lane, keeping those inside the
        // footprint.
        __shared__ const float* qleaf[kMajorantQueue];
        __shared__ int qblock[kMajorantQueue];
        __shared__ int qn;
        if (threadIdx.x == 0) qn = 0;
        __syncthreads();
        const int bx0 = x0 >> 3, by0 = y0 >> 3, bz0 = z0 >> 3;
        const int nbx = ((x0 + E - 1) >> 3) - bx0 + 1, nby = ((y0 + E - 1) >> 3) - by0 + 1,
                  nbz = ((z0 + E - 1) >> 3) - bz0 + 1;
        for (int b = threadIdx.x; b < nbx * nby * nbz; b += kBlock) {
            const int lx = bx0 + b % nbx, ly = by0 + (b / nbx) % nby, lz = bz0 + b / (nbx * nby);
            const LeafH h = acc.resolve(lx, ly, lz);
            if (h.m == 0u) {
                vmin = fminf(vmin, h.p[0]);
                vmax = fmaxf(vmax, h.p[0]);
            } else {
                const int q = atomicAdd(&qn, 1);
                qleaf[q] = h.p;
                qblock[q] = b;
            }
        }
        __syncthreads();
        const int lane = threadIdx.x & 63, nq = qn;
        for (int q = threadIdx.x >> 6; q < nq; q += kBlock / 64) {
            const int b = qblock[q];
            const int ox = 8 * (bx0 + b % nbx) - x0, oy = 8 * (by0 + (b / nbx) % nby) - y0,
                      oz = 8 * (bz0 + b / (nbx * nby)) - z0;
            const float* p = qleaf[q];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int n3 = lane + 64 * s;
                const int i = ox + (n3 & 7), j = oy + ((n3 >> 3) & 7), k = oz + (n3 >> 6);
                if ((unsigned)i < (unsigned)E && (unsigned)j < (unsigned)E && (unsigned)k < (unsigned)E) {
                    const float v = p[n3];
                    vmin = fminf(vmin, v);
                    vmax = fmaxf(vmax, v);
                }
            }
        }
    } else {
        for (int col = threadIdx.x; col < E * E; col += kBlock) {
            const int i = col % E, j = col / E;
            for (int k = 0; k < E; ++k) {
                const float v = acc.voxel(x0 + i, y0 + j, z0 + k);
                vmin = fminf(vmin, v);
                vmax = fmaxf(vmax, v);
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        vmin = fminf(vmin, __shfl_xor(vmin, o));
        vmax = fmaxf(vmax, __shfl_xor(vmax, o));
    }
    __shared__ float red[2][kBlock / 64];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = vmin;
        red[1][w] = vmax;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int q = 1; q < kBlock / 64; ++q) {
        vmin = fminf(vmin, red[0][q]);
        vmax = fmaxf(vmax, red[1][q]);
    }
    // max of the piecewise-linear alpha over [vmin, vmax]: the two ends and
    // every control point strictly inside
    float a = fmaxf(tf_alpha(m, vmin), tf_alpha(m, vmax));
    const float p0 = (vmin - m.tf_lo) * m.tf_inv, p1 = (vmax - m.tf_lo) * m.tf_inv;
    for (int q = 0; q < m.tf_n; ++q)
        if ((float)q > p0 && (float)q < p1) a = fmaxf(a, m.tf[q].w);
    out[cell] = m.ds * a;
}

template <class Acc, class View>
__global__ __launch_bounds__(kBlock) void majorant_kernel(View view, MediumK m, int C, int gx,
                                                          int gy, int gz, float* __restrict__ out)
{
    (void)gz;
    Acc acc{view};
    acc.reset();
    majorant_cell(acc, m, C, gx, gy, blockIdx.x, out);
}

// ---------------------------------------------------------------- EA

template <class Acc, class View, bool HDDA, bool COUNT>
__global__ __launch_bounds__(kBlock) void ea_kernel(View view, CameraK cam, MediumK m, float step,
                                                    float t_term, float* __restrict__ image,
                                                    unsigned long long* counter)
{
    Acc acc{view};
    acc.reset();
    int px, py;
    const bool live = tile_pixel(cam.width, cam.height, 8, blockIdx.x, blockIdx.y, px, py);
    uint32_t nsamp = 0;
    if (live) {
        float o[3], d[3], t0, t1;
        camera_ray(cam, (float)px + 0.5f, (float)py + 0.5f, o, d);
        float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, T = 1.0f;
        const float id[3] = {1.0f / d[0], 1.0f / d[1], 1.0f / d[2]};
        if (box_clip(view.nx, view.ny, view.nz, o, d, id, t0, t1)) {
            for (int k = 0;; ++k) {
                const float t = fmaf((float)k + 0.5f, step, t0);
                if (t >= t1) break;
                const float x = fmaf(t, d[0], o[0]), y = fmaf(t, d[1], o[1]),
                            z = fmaf(t, d[2], o[2]);
                if (HDDA) {
                    const int i = (int)floorf(fmaxf(x, -2.0f)), j = (int)floorf(fmaxf(y, -2.0f)),
                              kk = (int)floorf(fmaxf(z, -2.0f));
                    const int L = acc.in_stored_leaf(i, j, kk) ? 0 : acc.empty_level(i, j, kk);
                    if (L) {
                        const int mask = (1 << L) - 1;
                        if ((i & mask) != mask && (j & mask) != mask && (kk & mask) != mask) {
                            // every sample whose footprint stays inside this
                            // empty node reads B with alpha 0: jump past it
                            const int lo[3] = {i & ~mask, j & ~mask, kk & ~mask};
                            float te = INFINITY;
#pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                if (d[a] > 0.0f)
                                    te = fminf(te, ((float)(lo[a] + mask) - kHddaEps - o[a]) / d[a]);
                                else if (d[a] < 0.0f)
                                    te = fminf(te, ((float)lo[a] + kHddaEps - o[a]) / d[a]);
                            }
                            const int kn = (int)floorf(fminf((te - t0) / step - 0.5f, 2.0e9f));
                            k = (kn > k + 1 ? kn : k + 1) - 1;
                            continue;
                        }
                    }
                }
                const float s = trilinear(acc, x, y, z);
                if (COUNT) ++nsamp;
                const float4 c = tf_eval(m, s);
                const float a = 1.0f - expf(-(m.ds * c.w) * step);
                const float ta = T * a;
                c0 = fmaf(ta, c.x, c0);
                c1 = fmaf(ta, c.y, c1);
                c2 = fmaf(ta, c.z, c2);
                T *= 1.0f - a;
                if (T < t_term) break;
            }
        }
        float4* img = reinterpret_cast<float4*>(image);
        img[(uint64_t)py * cam.width + px] = make_float4(c0, c1, c2, 1.0f - T);
    }
    if (COUNT) block_count(nsamp, counter);
}

// ---------------------------------------------------------------- ISO

// Implicit iso-surface marcher (the interval-based marcher of Section 5.4):
// the EA lattice t0 + (k + 1/2) step, the first pair of consecutive samples
// on opposite sides of the iso value (side: f >= iso), `refine` bisection
// steps on that interval, normal -grad f / |grad f| by central differences
// of half a voxel.  With HDDA, lattice samples whose trilinear footprint lies
// inside an empty node read B at every corner, so they take B's side without
// a field read; the crossing, the bisection and the image are unchanged.
template <class Acc, class View, bool HDDA, bool COUNT>
__global__ __launch_bounds__(kBlock) void iso_kernel(View view, CameraK cam, float iso, float step,
                                                     int refine, float* __restrict__ image,
                                                     float* __restrict__ aov,
                                                     unsigned long long* counter)
{
    Acc acc{view};
    acc.reset();
    int px, py;
    const bool live = tile_pixel(cam.width, cam.height, 8, blockIdx.x, blockIdx.y, px, py);
    uint32_t nsamp = 0;
    if (live) {
        float o[3], d[3], t0, t1;
        camera_ray(cam, (float)px + 0.5f, (float)py + 0.5f, o, d);
        float4 out = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        float thit = -1.0f;
        const float id[3] = {1.0f / d[0], 1.0f / d[1], 1.0f / d[2]};
        if (box_clip(view.nx, view.ny, view.nz, o, d, id, t0, t1)) {
            const bool bg_side = acc.background() >= iso;
            bool have = false, prev = false;
            float tprev = 0.0f;
            for (int k = 0;; ++k) {
                const float t = fmaf((float)k + 0.5f, step, t0);
                if (t >= t1) break;
                const float x = fmaf(t, d[0], o[0]), y = fmaf(t, d[1], o[1]), z = fmaf(t, d[2], o[2]);
                bool side;
                int last = k;   // last lattice sample of this step
                bool skip = false;
                if (HDDA) {
                    const int i = (int)floorf(fmaxf(x, -2.0f)), j = (int)floorf(fmaxf(y, -2.0f)),
                              kk = (int)floorf(fmaxf(z, -2.0f));
                    const int L = acc.in_stored_leaf(i, j, kk) ? 0 : acc.empty_level(i, j, kk);
                    if (L) {
                        const int mask = (1 << L) - 1;
                        if ((i & mask) != mask && (j & mask) != mask && (kk & mask) != mask) {
                            const int lo[3] = {i & ~mask, j & ~mask, kk & ~mask};
                            float te = INFINITY;
#pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                if (d[a] > 0.0f)
                                    te = fminf(te, ((float)(lo[a] + mask) - kHddaEps - o[a]) / d[a]);
                                else if (d[a] < 0.0f)
                                    te = fminf(te, ((float)lo[a] + kHddaEps - o[a]) / d[a]);
                            }
                            const int kn = (int)floorf(fminf((te - t0) / step - 0.5f, 2.0e9f));
                            last = (kn > k + 1 ? kn : k + 1) - 1;
                            skip = true;
                        }
                    }
                }
                if (skip) {
                    side = bg_side;
                } else {
                    side = trilinear(acc, x, y, z) >= iso;
                    if (COUNT) ++nsamp;
                }
                if (have && side != prev) {
                    // `refine` bisection steps, then the six central-difference
                    // samples of the normal, through one field evaluation
                    float lo = tprev, hi = t, mid = 0.0f;
                    float p0 = 0.0f, p1 = 0.0f, p2 = 0.0f, gx = 0.0f, gy = 0.0f, gz = 0.0f;
                    for (int it = 0; it < refine + 6; ++it) {
                        float q0, q1, q2;
                        const int e = it - refine;   // >= 0: gradient sample e
                        if (e < 0) {
                            mid = 0.5f * (lo + hi);
                            q0 = fmaf(mid, d[0], o[0]);
                            q1 = fmaf(mid, d[1], o[1]);
                            q2 = fmaf(mid, d[2], o[2]);
                        } else {
                            if (e == 0) {
                                thit = 0.5f * (lo + hi);
                                p0 = fmaf(thit, d[0], o[0]);
                                p1 = fmaf(thit, d[1], o[1]);
                                p2 = fmaf(thit, d[2], o[2]);
                            }
                            const float sh = (e & 1) ? -0.5f : 0.5f;
                            q0 = p0 + ((e >> 1) == 0 ? sh : 0.0f);
                            q1 = p1 + ((e >> 1) == 1 ? sh : 0.0f);
                            q2 = p2 + ((e >> 1) == 2 ? sh : 0.0f);
                        }
                        const float w = trilinear(acc, q0, q1, q2);
                        if (COUNT) ++nsamp;
                        if (e < 0) {
                            if ((w >= iso) == prev) lo = mid;
                            else hi = mid;
                        } else {
                            const float sw = (e & 1) ? -w : w;
                            if ((e >> 1) == 0) gx += sw;
                            else if ((e >> 1) == 1) gy += sw;
                            else gz += sw;
                        }
                    }
                    const float len = sqrtf(gx * gx + gy * gy + gz * gz);
                    out = len > 0.0f ? make_float4(0.5f * (1.0f - gx / len), 0.5f * (1.0f - gy / len),
                                                   0.5f * (1.0f - gz / len), 1.0f)
                                     : make_float4(0.5f, 0.5f, 0.5f, 1.0f);
                    break;
                }
                have = true;
                prev = side;
                tprev = last == k ? t : fmaf((float)last + 0.5f, step, t0);
                k = last;
            }
        }
        const uint64_t pix = (uint64_t)py * cam.width + px;
        reinterpret_cast<float4*>(image)[pix] = out;
        if (aov) reinterpret_cast<float2*>(aov)[pix] = make_float2(thit, 0.0f);
    }
    if (COUNT) block_count(nsamp, counter);
}

// ---------------------------------------------------------------- host side

static vdbc_status make_medium(const vdbc_medium* m, int nx, int ny, int nz, MediumK* k)
{
    if (!m) return fail(VDBC_E_INVALID, "null medium");
    if (m->tf_n < 2 || m->tf_n > 64) return fail(VDBC_E_INVALID, "tf_n must be in [2, 64]");
    if (!(m->tf_hi > m->tf_lo) || !std::isfinite(m->tf_lo) || !std::isfinite(m->tf_hi))
        return fail(VDBC_E_INVALID, "need finite tf_lo < tf_hi");
    if (!std::isfinite(m->sigma_scale) || m->sigma_scale < 0.0f)
        return fail(VDBC_E_INVALID, "sigma_scale must be finite and >= 0");
    std::memset(k, 0, sizeof *k);
    const int nmax = nx > ny ? (nx > nz ? nx : nz) : (ny > nz ? ny : nz);
    k->ds = m->sigma_scale / (float)nmax;
    k->albedo = m->albedo;
    k->tf_n = (int)m->tf_n;
    k->tf_lo = m->tf_lo;
    k->tf_inv = (float)(m->tf_n - 1) / (m->tf_hi - m->tf_lo);
    for (uint32_t i = 0; i < m->tf_n; ++i) {
        for (int c = 0; c < 4; ++c)
            if (!std::isfinite(m->tf[i][c])) return fail(VDBC_E_INVALID, "non-finite TF entry");
        if (m->tf[i][3] < 0.0f) return fail(VDBC_E_INVALID, "TF alpha must be >= 0");
        k->tf[i] = make_float4(m->tf[i][0], m->tf[i][1], m->tf[i][2], m->tf[i][3]);
    }
    for (int a = 0; a < 3; ++a) {
        k->light[a] = m->light_dir[a];
        k->light_E[a] = m->light_E[a];
        k->ambient[a] = m->ambient[a];
    }
    if (m->env) {
        if (m->env_w == 0 || m->env_h == 0 || (uint64_t)m->env_w * m->env_h > (1ull << 28))
            return fail(VDBC_E_INVALID, "env map needs 1 <= env_w * env_h <= 2^28 texels");
        k->env = m->env;
        k->env_w = (int)m->env_w;
        k->env_h = (int)m->env_h;
    }
    return VDBC_OK;
}

// Host mirror of the device TF alpha (for the HDDA precondition alpha(B)=0).
static float host_alpha(const MediumK& m, float s)
{
    float pos = (s - m.tf_lo) * m.tf_inv;
    pos = std::fmin(std::fmax(pos, 0.0f), (float)(m.tf_n - 1));
    int i = (int)pos;
    i = i > m.tf_n - 2 ? m.tf_n - 2 : i;
    const float fr = pos - (float)i;
    return std::fma(fr, m.tf[i + 1].w - m.tf[i].w, m.tf[i].w);
}

static vdbc_status make_camera(const vdbc_camera* c, CameraK* k)
{
    if (!c) return fail(VDBC_E_INVALID, "null camera");
    if (c->kind > 1) return fail(VDBC_E_INVALID, "camera kind must be 0 or 1");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(c->origin[a]) || !std::isfinite(c->lower_left[a]) ||
            !std::isfinite(c->du[a]) || !std::isfinite(c->dv[a]) || !std::isfinite(c->dir[a]))
            return fail(VDBC_E_INVALID, "non-finite camera vector");
    if (c->kind == 0 && c->dir[0] == 0.0f && c->dir[1] == 0.0f && c->dir[2] == 0.0f)
        return fail(VDBC_E_INVALID, "orthographic camera needs a non-zero direction");
    if (c->width == 0 || c->height == 0 || c->width > 65536 * kTile || c->height > 65535u * kTile ||
        (uint64_t)c->width * c->height > (1ull << 31))
        return fail(VDBC_E_INVALID, "bad image size (1..2^31 pixels)");
    k->kind = (int)c->kind;
    k->width = (int)c->width;
    k->height = (int)c->height;
    for (int a = 0; a < 3; ++a) {
        k->o[a] = c->origin[a];
        k->ll[a] = c->lower_left[a];
        k->du[a] = c->du[a];
        k->dv[a] = c->dv[a];
        k->dir[a] = c->dir[a];
    }
    return VDBC_OK;
}

static uint64_t majorant_bytes(uint32_t C, int nx, int ny, int nz)
{
    const uint64_t gx = (nx + C - 1) / C, gy = (ny + C - 1) / C, gz = (nz + C - 1) / C;
    return gx * gy * gz * 4u;
}

// Majorant grid and coarse occupancy geometry.  Coarse blocks are 2^lf
// macrocells per axis, the largest power of two spanning at most 64 voxels
// (2^3 bricks), doubled until the bit mask fits in 32 KB of LDS.
static void pt_geometry(uint32_t C, int nx, int ny, int nz, PtArgs* g)
{
    g->C = (int)C;
    g->invC = 1.0f / (float)C;
    g->gx = (nx + g->C - 1) / g->C;
    g->gy = (ny + g->C - 1) / g->C;
    g->gz = (nz + g->C - 1) / g->C;
    int lf = 0;
    // coarse blocks of at least 4 macrocells and at least 64 voxels per axis
    // (64 voxels up to C = 16, 4 cells from there on)
    const uint32_t edge = std::max<uint32_t>(64u, 4u * C);
    while ((C << (lf + 1)) <= edge) ++lf;
    for (;;) {
        const int F = 1 << lf;
        g->lf = lf;
        g->cgx = (g->gx + F - 1) / F;
        g->cgy = (g->gy + F - 1) / F;
        g->cgz = (g->gz + F - 1) / F;
        const uint64_t cells = (uint64_t)g->cgx * g->cgy * g->cgz;
        g->cwords = (int)((cells + 31) / 32);
        if (g->cwords <= 8192) break;
        ++lf;
    }
}

static uint64_t pt_workspace(uint32_t C, int nx, int ny, int nz)
{
    PtArgs g;
    pt_geometry(C, nx, ny, nz, &g);
    return 256 + align256(majorant_bytes(C, nx, ny, nz)) + align256(4ull * g.cwords);
}

// A path-traced launch splits its tiles into several work items (and needs
// the per-pixel sums after the occupancy bits) iff 0 < chunk_spp < spp.
static bool pt_split(const vdbc_render_params* r) { return r->chunk_spp != 0 && r->chunk_spp < r->spp; }

// Bytes of the per-pixel sums of a split launch: 32 (red, green, blue,
// hits | escapes) + 8 (AOV depth) per pixel.
static uint64_t pt_sums_bytes(uint64_t npix) { return align256(40ull * npix); }

// 256-pixel tiles of a path-traced image: 4 tw x 64 / tw pixels each.
static uint64_t pt_tiles_x(uint64_t width, uint64_t tw) { return (width + 4 * tw - 1) / (4 * tw); }
static uint64_t pt_tiles(uint64_t width, uint64_t height, uint64_t tw)
{
    return pt_tiles_x(width, tw) * ((height + 64 / tw - 1) / (64 / tw));
}

// Bytes of the cost order (VDBC_RENDER_COST_ORDER): bin histogram and bin
// offsets (kCostBins u32 each), then per tile its bin and its place in the
// order (u32 each).
static uint64_t pt_order_bytes(uint64_t tiles) { return align256(8ull * kCostBins + 8ull * tiles); }


template <class Acc, class View>
static vdbc_status launch_majorant(const View& v, const MediumK& m, uint32_t C, float* out,
                                   hipStream_t st)
{
    const int gx = (v.nx + C - 1) / C, gy = (v.ny + C - 1) / C, gz = (v.nz + C - 1) / C;
    const uint64_t cells = (uint64_t)gx * gy * gz;
    if (C < 4 || C > 64) return fail(VDBC_E_INVALID, "macrocell must be in [4, 64]");   // sizes kMajorantQueue
    if (cells > 0x7FFFFFFFull) return fail(VDBC_E_INVALID, "too many macrocells (%llu)", (unsigned long long)cells);
    hipLaunchKernelGGL((majorant_kernel<Acc, View>), dim3((unsigned)cells), dim3(kBlock), 0, st, v, m,
                       (int)C, gx, gy, gz, out);
    return launch_check("majorant");
}

// Compute units of the current device (cached per device; 256 if unknown).
static int device_cus()
{
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 256;
    if (dev < 64 && cache[dev].load(std::memory_order_relaxed) > 0)
        return cache[dev].load(std::memory_order_relaxed);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    if (dev < 64) cache[dev].store(cus, std::memory_order_relaxed);
    return cus;
}

// MARCH = false leaves out the EA and ISO kernels (accessor variants that
// only the path tracer uses).
template <class Acc, class View, bool MARCH = true>
static vdbc_status render_impl(const View& v, const vdbc_camera* c, const vdbc_medium* med,
                               const vdbc_render_params* r, float* image, float* aov, void* ws,
                               uint64_t ws_bytes, void* stream)
{
    if (!r || !image) return fail(VDBC_E_INVALID, "null params or image");
    CameraK cam;
    MediumK m;
    vdbc_status s = make_camera(c, &cam);
    if (s) return s;
    if (r->mode > 2) return fail(VDBC_E_INVALID, "mode must be EA (0), PT (1) or ISO (2)");
    if (r->mode != VDBC_MODE_ISO) {
        s = make_medium(med, v.nx, v.ny, v.nz, &m);
        if (s) return s;
    }
    const bool count = (r->flags & VDBC_RENDER_COUNT) != 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned long long* counter = reinterpret_cast<unsigned long long*>(ws);
    vdbc_dims d{(uint32_t)v.nx, (uint32_t)v.ny, (uint32_t)v.nz};
    uint64_t need = 0;
    s = vdbc_render_workspace(r, d, c, &need);
    if (s) return s;
    if (need && (!ws || ws_bytes < need))
        return fail(VDBC_E_BUFFER_TOO_SMALL, "workspace needs %llu bytes", (unsigned long long)need);
    if (ws && reinterpret_cast<uintptr_t>(ws) % 256)
        return fail(VDBC_E_INVALID, "workspace must be 256-byte aligned");
    dim3 grid((cam.width + kTile - 1) / kTile, (cam.height + kTile - 1) / kTile);
    if constexpr (MARCH) {
        if (r->mode == VDBC_MODE_ISO) {
            if (!(r->step > 0.0f) || !std::isfinite(r->step))
                return fail(VDBC_E_INVALID, "ISO step must be finite and > 0");
            const double diag = std::sqrt((double)v.nx * v.nx + (double)v.ny * v.ny + (double)v.nz * v.nz);
            if (diag / r->step > 16777216.0)
                return fail(VDBC_E_INVALID, "ISO step too small for this volume (> 2^24 samples per ray)");
            if (!std::isfinite(r->iso)) return fail(VDBC_E_INVALID, "iso value must be finite");
            if (r->refine > 64) return fail(VDBC_E_INVALID, "refine must be <= 64");
            if (count) {
                hipLaunchKernelGGL(zero_u64, dim3(1), dim3(64), 0, st, counter);
                if ((s = launch_check("zero counter"))) return s;
            }
            const bool hdda = (r->flags & VDBC_RENDER_HDDA) != 0;
    #define ISO_LAUNCH(H, CNT)                                                                      \
        hipLaunchKernelGGL((iso_kernel<Acc, View, H, CNT>), grid, dim3(kBlock), 0, st, v, cam, r->iso, \
                           r->step, (int)r->refine, image, aov, counter)
            if (hdda) {
                if (count) ISO_LAUNCH(true, true);
                else ISO_LAUNCH(true, false);
            } else {
                if (count) ISO_LAUNCH(false, true);
                else ISO_LAUNCH(false, false);
            }
    #undef ISO_LAUNCH
            return launch_check("iso render");
        }
        if (count && r->mode == VDBC_MODE_EA) {
            hipLaunchKernelGGL(zero_u64, dim3(1), dim3(64), 0, st, counter);
            if ((s = launch_check("zero counter"))) return s;
        }
        if (r->mode == VDBC_MODE_EA) {
            if (!(r->step > 0.0f) || !std::isfinite(r->step))
                return fail(VDBC_E_INVALID, "EA step must be finite and > 0");
            // bound the per-ray loop: box diagonal / step <= 2^24 samples
            const double diag = std::sqrt((double)v.nx * v.nx + (double)v.ny * v.ny + (double)v.nz * v.nz);
            if (diag / r->step > 16777216.0)
                return fail(VDBC_E_INVALID, "EA step too small for this volume (> 2^24 samples per ray)");
            const bool hdda = (r->flags & VDBC_RENDER_HDDA) && host_alpha(m, v.background) == 0.0f;
    #define EA_LAUNCH(H, CNT)                                                                      \
        hipLaunchKernelGGL((ea_kernel<Acc, View, H, CNT>), grid, dim3(kBlock), 0, st, v, cam, m, \
                           r->step, r->t_terminate, image, counter)
            if (hdda) {
                if (count) EA_LAUNCH(true, true);
                else EA_LAUNCH(true, false);
            } else {
                if (count) EA_LAUNCH(false, true);
                else EA_LAUNCH(false, false);
            }
    #undef EA_LAUNCH
            return launch_check("ea render");
        }
    } else if (r->mode != VDBC_MODE_PT) {
        return fail(VDBC_E_UNSUPPORTED, "accessor variant for the path tracer only");
    }
    // the tile's work units (256 x spp) are 32-bit and the bounce is a
    // 16-bit field of the random-number counter
    if (r->spp == 0 || r->spp > kMaxSpp || r->max_bounces == 0 || r->max_bounces > kMaxBounces)
        return fail(VDBC_E_INVALID, "need 1 <= spp <= %u and 1 <= max_bounces <= %u", kMaxSpp, kMaxBounces);
    if (r->tile_w != 0 && r->tile_w != 8 && r->tile_w != 16 && r->tile_w != 32 && r->tile_w != 64)
        return fail(VDBC_E_INVALID, "tile_w must be 0 (default 8), 8, 16, 32 or 64");
    {
        // the work-item queue counts in 32 bits
        const uint64_t tiles = pt_tiles((uint64_t)cam.width, (uint64_t)cam.height, r->tile_w == 0 ? 8 : r->tile_w);
        const uint64_t per_tile = pt_split(r) ? (r->spp + r->chunk_spp - 1) / r->chunk_spp : 1;
        if (tiles * per_tile > 0xFFFFFFFFull)
            return fail(VDBC_E_INVALID, "more than 2^32 work items: raise chunk_spp");
    }
    {
        const double l = std::sqrt((double)med->light_dir[0] * med->light_dir[0] +
                                   (double)med->light_dir[1] * med->light_dir[1] +
                                   (double)med->light_dir[2] * med->light_dir[2]);
        if (!(std::fabs(l - 1.0) <= 1e-3)) return fail(VDBC_E_INVALID, "light_dir must be a unit vector");
        if (!std::isfinite(med->albedo) || med->albedo < 0.0f)
            return fail(VDBC_E_INVALID, "albedo must be finite and >= 0");
    }
    hipLaunchKernelGGL(zero_u64, dim3(1), dim3(64), 0, st, counter);   // counters and tile queue
    if ((s = launch_check("zero counters"))) return s;
    float* maj = reinterpret_cast<float*>(static_cast<uint8_t*>(ws) + 256);
    if (!(r->flags & VDBC_RENDER_KEEP_MAJORANT)) {
        s = launch_majorant<Acc>(v, m, r->macrocell, maj, st);
        if (s) return s;
    }
    PtArgs g;
    pt_geometry(r->macrocell, v.nx, v.ny, v.nz, &g);
    g.spp = (int)r->spp;
    g.max_bounces = (int)r->max_bounces;
    g.tw = r->tile_w == 0 ? 8 : (int)r->tile_w;
    g.seed_lo = (uint32_t)r->seed;
    g.seed_hi = (uint32_t)(r->seed >> 32);
    g.frame = r->frame;
    g.rr = (r->flags & VDBC_RENDER_RR) ? 1 : 0;
    const bool split = pt_split(r);
    g.chunk = split ? r->chunk_spp : r->spp;
    g.chunks = (r->spp + g.chunk - 1) / g.chunk;
    uint32_t* coarse = reinterpret_cast<uint32_t*>(
        static_cast<uint8_t*>(ws) + 256 + align256(majorant_bytes(r->macrocell, v.nx, v.ny, v.nz)));
    const uint64_t npix = (uint64_t)cam.width * (uint64_t)cam.height;
    const uint64_t tiles = pt_tiles((uint64_t)cam.width, (uint64_t)cam.height, (uint64_t)g.tw);
    uint8_t* const tail = static_cast<uint8_t*>(ws) + pt_workspace(r->macrocell, v.nx, v.ny, v.nz);
    PtSums sums{};
    if (split) {
        uint8_t* base = tail;
        sums.rgbn = reinterpret_cast<unsigned long long*>(base);
        sums.depth = sums.rgbn + 4 * npix;
        const uint64_t words = pt_sums_bytes(npix) / 16;
        hipLaunchKernelGGL(pt_sums_clear_kernel, dim3((unsigned)std::min<uint64_t>((words + kBlock - 1) / kBlock, 4096)),
                           dim3(kBlock), 0, st, reinterpret_cast<uint4*>(base), words);
        if ((s = launch_check("clear pixel sums"))) return s;
    }
    {
        const uint64_t ncoarse = (uint64_t)g.cgx * g.cgy * g.cgz;
        hipLaunchKernelGGL(coarse_bits_kernel, dim3((unsigned)((ncoarse + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, st, maj, g, coarse);
        if ((s = launch_check("coarse occupancy"))) return s;
    }
    const uint32_t* order = nullptr;
    if (r->flags & VDBC_RENDER_COST_ORDER) {
        uint32_t* hist = reinterpret_cast<uint32_t*>(tail + (split ? pt_sums_bytes(npix) : 0));
        uint32_t* off = hist + kCostBins;
        uint32_t* key = off + kCostBins;
        uint32_t* ord = key + tiles;
        const unsigned tb = (unsigned)((tiles + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(pt_sums_clear_kernel, dim3(1), dim3(kBlock), 0, st, reinterpret_cast<uint4*>(hist),
                           (uint64_t)(2 * kCostBins / 4));
        hipLaunchKernelGGL(pt_tile_cost_kernel, dim3(tb), dim3(kBlock), 0, st, cam, g, v.nx, v.ny, v.nz, maj,
                           (uint32_t)pt_tiles_x((uint64_t)cam.width, (uint64_t)g.tw), (uint32_t)tiles, key, hist);
        hipLaunchKernelGGL(pt_cost_offsets_kernel, dim3(1), dim3(64), 0, st, hist, off);
        hipLaunchKernelGGL(pt_cost_scatter_kernel, dim3(tb), dim3(kBlock), 0, st, key, off, ord, (uint32_t)tiles);
        if ((s = launch_check("cost order"))) return s;
        order = ord;
    }
    const size_t lds = 4u * (size_t)g.cwords;
    grid = dim3((unsigned)std::min<uint64_t>(tiles * g.chunks, (uint64_t)device_cus() * kPtBlocksPerCu));
    uint32_t* queue = reinterpret_cast<uint32_t*>(counter + 2);
#define PT_LAUNCH(CNT, AO, EN)                                                                     \
    hipLaunchKernelGGL((pt_kernel<Acc, View, CNT, AO, EN>), grid, dim3(kBlock), lds, st, v, cam, m, \
                       g, maj, coarse, image, aov, counter, queue, sums, order)
#define PT_LAUNCH_ENV(CNT, AO)           \
    if (m.env) PT_LAUNCH(CNT, AO, true); \
    else PT_LAUNCH(CNT, AO, false)
    if (count) {
        if (aov) PT_LAUNCH_ENV(true, true);
        else PT_LAUNCH_ENV(true, false);
    } else {
        if (aov) PT_LAUNCH_ENV(false, true);
        else PT_LAUNCH_ENV(false, false);
    }
#undef PT_LAUNCH_ENV
#undef PT_LAUNCH
    if (split) {
        if ((s = launch_check("pt render"))) return s;
        hipLaunchKernelGGL(pt_resolve_kernel, dim3((unsigned)((npix + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, sums,
                           image, aov, (uint32_t)npix, g.spp);
        return launch_check("pixel sums to image");
    }
    return launch_check("pt render");
}

}  // namespace vdbc

using namespace vdbc;

extern "C" vdbc_status vdbc_render_workspace(const vdbc_render_params* r, vdbc_dims d,
                                             const vdbc_camera* c, uint64_t* bytes)
{
    if (!r || !bytes) return fail(VDBC_E_INVALID, "null argument");
    if (d.nx == 0 || d.ny == 0 || d.nz == 0) return fail(VDBC_E_INVALID, "zero dims");
    if (r->mode == VDBC_MODE_PT) {
        if (r->macrocell < 4 || r->macrocell > 64 || (r->macrocell & (r->macrocell - 1)))
            return fail(VDBC_E_INVALID, "macrocell must be 4, 8, 16, 32 or 64");
        *bytes = pt_workspace(r->macrocell, (int)d.nx, (int)d.ny, (int)d.nz);
        if (pt_split(r)) {
            if (!c) return fail(VDBC_E_INVALID, "0 < chunk_spp < spp: the workspace size needs the camera");
            *bytes += pt_sums_bytes((uint64_t)c->width * (uint64_t)c->height);
        }
        if (r->flags & VDBC_RENDER_COST_ORDER) {
            if (!c) return fail(VDBC_E_INVALID, "VDBC_RENDER_COST_ORDER: the workspace size needs the camera");
            if (r->tile_w != 0 && r->tile_w != 8 && r->tile_w != 16 && r->tile_w != 32 && r->tile_w != 64)
                return fail(VDBC_E_INVALID, "tile_w must be 0 (default 8), 8, 16, 32 or 64");
            *bytes += pt_order_bytes(pt_tiles(c->width, c->height, r->tile_w == 0 ? 8 : r->tile_w));
        }
    } else {
        *bytes = (r->flags & VDBC_RENDER_COUNT) ? 256 : 0;
    }
    return VDBC_OK;
}

static vdbc_status render_vdb(const vdbc_grid* g, const vdbc_camera* c, const vdbc_medium* m,
                              const vdbc_render_params* r, float* image, float* aov, void* ws,
                              uint64_t ws_bytes, void* stream)
{
    VdbView v;
    vdbc_status s = make_view(g, &v);
    if (s) return s;
    // path tracer only: the accessor's cache policy (a tuning knob; the image
    // does not depend on it)
    const uint32_t pol = r ? (r->flags & (VDBC_RENDER_CACHE_NONE | VDBC_RENDER_CACHE_LEAF)) : 0u;
    if (pol == (VDBC_RENDER_CACHE_NONE | VDBC_RENDER_CACHE_LEAF))
        return fail(VDBC_E_INVALID, "at most one cache-policy flag");
    if (pol && r->mode == VDBC_MODE_PT) {
        if (pol == VDBC_RENDER_CACHE_NONE)
            return render_impl<VdbAccT<kCacheNone>, VdbView, false>(v, c, m, r, image, aov, ws, ws_bytes, stream);
        return render_impl<VdbAccT<kCacheLeaf>, VdbView, false>(v, c, m, r, image, aov, ws, ws_bytes, stream);
    }
    return render_impl<VdbAcc>(v, c, m, r, image, aov, ws, ws_bytes, stream);
}

extern "C" vdbc_status vdbc_render(const vdbc_grid* g, const vdbc_camera* c, const vdbc_medium* m,
                                   const vdbc_render_params* r, float* image, float* aov, void* ws,
                                   uint64_t ws_bytes, void* stream)
{
    clear_error();
    return render_vdb(g, c, m, r, image, aov, ws, ws_bytes, stream);
}

// ---------------------------------------------------------------- render without allocation

// Fixed scratch of vdbc_render_noalloc: the render workspace (counters, tile
// queue, majorant grid, coarse occupancy bits) of one call.  Every GPU the
// library runs on holds its own copy until the process ends.  Host code never
// passes the symbol itself to a kernel: it takes the device address that
// hipGetSymbolAddress returns for the current device.
constexpr uint64_t kScratchBytes = VDBC_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) uint8_t scratch[kScratchBytes];

// Device address of `scratch` on the current device, resolved once per
// device (with that device current) on its first call.
static vdbc_status scratch_address(void** out)
{
    static std::mutex mu;
    static void* addr[64] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(VDBC_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= 64) return fail(VDBC_E_UNSUPPORTED, "device index %d beyond 63", dev);
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(VDBC_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                        hipGetErrorString(e));
        addr[dev] = p;
    }
    *out = addr[dev];
    return VDBC_OK;
}

extern "C" vdbc_status vdbc_render_noalloc(const vdbc_grid* g, const vdbc_camera* c,
                                           const vdbc_medium* m, const vdbc_render_params* r,
                                           float* image, float* aov, void* stream)
{
    clear_error();
    if (!g || !r) return fail(VDBC_E_INVALID, "null grid or params");
    if (r->flags & VDBC_RENDER_KEEP_MAJORANT)
        return fail(VDBC_E_INVALID, "VDBC_RENDER_KEEP_MAJORANT: the scratch holds no majorant of the caller's");
    VdbView v;
    vdbc_status s = make_view(g, &v);
    if (s) return s;
    vdbc_dims d{(uint32_t)v.nx, (uint32_t)v.ny, (uint32_t)v.nz};
    uint64_t need = 0;
    if ((s = vdbc_render_workspace(r, d, c, &need))) return s;
    if (need > kScratchBytes)
        return fail(VDBC_E_BUFFER_TOO_SMALL, "this render needs %llu bytes of scratch; the fixed scratch holds %llu "
                    "(use vdbc_render with a workspace, a larger macrocell or chunk_spp 0)",
                    (unsigned long long)need, (unsigned long long)kScratchBytes);
    void* ws = nullptr;
    if ((s = scratch_address(&ws))) return s;
    return render_vdb(g, c, m, r, image, aov, ws, kScratchBytes, stream);
}

extern "C" vdbc_status vdbc_render_dense(const float* dense, vdbc_dims d, float background,
                                         const vdbc_camera* c, const vdbc_medium* m,
                                         const vdbc_render_params* r, float* image, float* aov,
                                         void* ws, uint64_t ws_bytes, void* stream)
{
    clear_error();
    DenseView v;
    vdbc_status s = make_dense(dense, d, background, &v);
    if (s) return s;
    return render_impl<DenseAcc>(v, c, m, r, image, aov, ws, ws_bytes, stream);
}

extern "C" vdbc_status vdbc_majorant(const vdbc_grid* g, const vdbc_medium* med, uint32_t C,
                                     float* out, void* stream)
{
    clear_error();
    VdbView v;
    vdbc_status s = make_view(g, &v);
    if (s) return s;
    if (!out) return fail(VDBC_E_INVALID, "null output");
    if (C < 4 || C > 64) return fail(VDBC_E_INVALID, "macrocell must be in [4, 64]");
    MediumK m;
    if ((s = make_medium(med, v.nx, v.ny, v.nz, &m))) return s;
    return launch_majorant<VdbAcc>(v, m, C, out, static_cast<hipStream_t>(stream));
}

extern "C" vdbc_status vdbc_majorant_dense(const float* dense, vdbc_dims d, float background,
                                           const vdbc_medium* med, uint32_t C, float* out,
                                           void* stream)
{
    clear_error();
    DenseView v;
    vdbc_status s = make_dense(dense, d, background, &v);
    if (s) return s;
    if (!out) return fail(VDBC_E_INVALID, "null output");
    if (C < 4 || C > 64) return fail(VDBC_E_INVALID, "macrocell must be in [4, 64]");
    MediumK m;
    if ((s = make_medium(med, v.nx, v.ny, v.nz, &m))) return s;
    return launch_majorant<DenseAcc>(v, m, C, out, static_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------- batched majorants
// The majorant grids and the coarse occupancy bits of every volume of a batch
// in one launch each, with the per-cell code of the single-volume kernels (so
// the grids and bits are bitwise those of per-volume launches): workgroup b
// belongs to the volume v with base[v] <= b < base[v + 1], a prefix table of
// the volumes' macrocells (coarse-bit workgroups), and works on its local
// index b - base[v].  Small volumes no longer leave the chip idle one launch
// at a time.

namespace vdbc {

__device__ inline uint32_t batch_volume_of(const uint32_t* __restrict__ base, uint32_t n, uint32_t b)
{
    uint32_t lo = 0, hi = n;   // base[lo] <= b < base[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (base[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void majorant_batch_kernel(const BatchDesc* __restrict__ descs,
                                                                const uint32_t* __restrict__ base, uint32_t n)
{
    __shared__ uint32_t s_v;
    if (threadIdx.x == 0) s_v = batch_volume_of(base, n, blockIdx.x);
    __syncthreads();
    const uint32_t v = s_v;
    const BatchDesc* D = descs + v;
    VdbAcc acc{D->view};
    acc.reset();
    majorant_cell(acc, D->med, D->g.C, D->g.gx, D->g.gy, blockIdx.x - base[v], const_cast<float*>(D->maj));
}

__global__ __launch_bounds__(kBlock) void coarse_bits_batch_kernel(const BatchDesc* __restrict__ descs,
                                                                   const uint32_t* __restrict__ base, uint32_t n)
{
    // every thread finds the volume itself: a workgroup lies in one volume,
    // and no barrier is needed before the ballot
    const uint32_t v = batch_volume_of(base, n, blockIdx.x);
    const BatchDesc* D = descs + v;
    coarse_bits_block(D->maj, D->g, const_cast<uint32_t*>(D->coarse), blockIdx.x - base[v]);
}

}  // namespace vdbc

// ---------------------------------------------------------------- batched PT (host)

struct vdbc_batch {
    uint32_t n = 0;
    vdbc_tuning t{};
    std::vector<VdbView> views;
    std::vector<CameraK> cams;
    std::vector<MediumK> meds;
    std::vector<PtArgs> gs;
    std::vector<float*> majs;
    std::vector<uint32_t*> coarse;
    std::vector<float*> images;
    std::vector<PtSums> sums;          // per volume: pixel sums of split items, or null
    std::vector<int> tiles_x, tiles_y;
    BatchDesc* d_descs = nullptr;
    uint32_t* d_items = nullptr;
    uint32_t* d_counter = nullptr;
    uint32_t* d_cell_base = nullptr;     // prefix tables of macrocells and coarse-bit workgroups
    uint32_t* d_coarse_base = nullptr;
    uint64_t cells_total = 0, cblocks_total = 0;
    uint32_t n_items = 0;
    int max_cwords = 0;
    int grid_blocks = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace vdbc {

static vdbc_status batch_tuning(const vdbc_tuning* t, vdbc_tuning* out)
{
    vdbc_tuning d{16, 8, 4, 1, 0};
    if (t) d = *t;
    if (d.macrocell < 4 || d.macrocell > 64 || (d.macrocell & (d.macrocell - 1)))
        return fail(VDBC_E_INVALID, "tuning.macrocell must be 4, 8, 16, 32 or 64");
    if (d.tile_w == 0) d.tile_w = 8;
    if (d.tile_w != 8 && d.tile_w != 16 && d.tile_w != 32 && d.tile_w != 64)
        return fail(VDBC_E_INVALID, "tuning.tile_w must be 8, 16, 32 or 64");
    if (d.blocks_per_cu == 0) d.blocks_per_cu = 4;
    if (d.blocks_per_cu > 32) return fail(VDBC_E_INVALID, "tuning.blocks_per_cu must be <= 32");
    *out = d;
    return VDBC_OK;
}

// Bytes of a batch volume's pixel sums (32 per pixel: RGB and the hit and
// escape counts; the batched launch writes no depth).
static uint64_t batch_sums_bytes(uint64_t npix) { return align256(32ull * npix); }

// Validates the items and fills the per-volume launch state; the offsets
// receive the workspace layout (counter, descriptors, item list, then per
// volume majorant, coarse bits and, for a split volume, its pixel sums; 0 for
// a volume that is not split) and the total size.
static vdbc_status batch_plan(const vdbc_batch_item* items, uint32_t n, const vdbc_tuning& t, vdbc_batch* b,
                              std::vector<uint64_t>* maj_off, std::vector<uint64_t>* coarse_off,
                              std::vector<uint64_t>* sums_off, uint64_t* items_off, uint64_t* total)
{
    if (!items || n == 0 || n > 4096) return fail(VDBC_E_INVALID, "need 1..4096 batch items");
    b->n = n;
    b->t = t;
    uint64_t tiles_total = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const vdbc_batch_item& it = items[i];
        VdbView v;
        CameraK cam;
        MediumK m;
        vdbc_status s = make_view(&it.grid, &v);
        if (!s) s = make_camera(&it.camera, &cam);
        if (!s) s = make_medium(&it.medium, v.nx, v.ny, v.nz, &m);
        if (s) return fail(s, "batch item %u: %s", i, vdbc_last_error());
        if (it.spp == 0 || it.spp > kMaxSpp || it.max_bounces == 0 || it.max_bounces > kMaxBounces || !it.image)
            return fail(VDBC_E_INVALID, "batch item %u: need 1 <= spp <= %u, 1 <= max_bounces <= %u and an image", i,
                        kMaxSpp, kMaxBounces);
        const double l = std::sqrt((double)it.medium.light_dir[0] * it.medium.light_dir[0] +
                                   (double)it.medium.light_dir[1] * it.medium.light_dir[1] +
                                   (double)it.medium.light_dir[2] * it.medium.light_dir[2]);
        if (!(std::fabs(l - 1.0) <= 1e-3)) return fail(VDBC_E_INVALID, "batch item %u: light_dir not unit", i);
        PtArgs g;
        pt_geometry(t.macrocell, v.nx, v.ny, v.nz, &g);
        g.spp = (int)it.spp;
        g.max_bounces = (int)it.max_bounces;
        g.tw = (int)t.tile_w;
        g.seed_lo = (uint32_t)it.seed;
        g.seed_hi = (uint32_t)(it.seed >> 32);
        g.frame = it.frame;
        g.rr = 0;
        const bool split = t.chunk_spp != 0 && t.chunk_spp < it.spp;
        g.chunk = split ? t.chunk_spp : (uint32_t)g.spp;
        g.chunks = split ? (it.spp + t.chunk_spp - 1) / t.chunk_spp : 1u;
        const int tx = (int)pt_tiles_x((uint64_t)cam.width, (uint64_t)g.tw),
                  ty = (int)(pt_tiles((uint64_t)cam.width, (uint64_t)cam.height, (uint64_t)g.tw) / (uint64_t)tx);
        if ((uint64_t)tx * ty * g.chunks > 0xFFFFFu)
            return fail(VDBC_E_INVALID, "batch item %u: image too large for %u work items per tile", i, g.chunks);
        b->views.push_back(v);
        b->cams.push_back(cam);
        b->meds.push_back(m);
        b->gs.push_back(g);
        b->images.push_back(it.image);
        b->tiles_x.push_back(tx);
        b->tiles_y.push_back(ty);
        tiles_total += (uint64_t)tx * ty * g.chunks;
        b->max_cwords = std::max(b->max_cwords, g.cwords);
    }
    uint64_t o = 256;                                   // counter
    const uint64_t descs_off = o;
    o += align256((uint64_t)n * sizeof(BatchDesc));
    o += align256(8ull * (n + 1));                      // the two prefix tables of the batched majorants
    *items_off = o;
    o += align256(tiles_total * 4);
    for (uint32_t i = 0; i < n; ++i) {
        maj_off->push_back(o);
        o += align256(majorant_bytes(t.macrocell, b->views[i].nx, b->views[i].ny, b->views[i].nz));
        coarse_off->push_back(o);
        o += align256(4ull * b->gs[i].cwords);
        if (b->gs[i].chunks > 1) {
            sums_off->push_back(o);
            o += batch_sums_bytes((uint64_t)b->cams[i].width * b->cams[i].height);
        } else {
            sums_off->push_back(0);
        }
    }
    (void)descs_off;
    b->n_items = (uint32_t)tiles_total;
    *total = o;
    return VDBC_OK;
}

// The images of the split volumes from their pixel sums.
static vdbc_status batch_resolve(vdbc_batch* b, hipStream_t st)
{
    for (uint32_t i = 0; i < b->n; ++i) {
        if (!b->sums[i].rgbn) continue;
        const uint64_t npix = (uint64_t)b->cams[i].width * b->cams[i].height;
        hipLaunchKernelGGL(pt_resolve_kernel, dim3((unsigned)((npix + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                           b->sums[i], b->images[i], nullptr, (uint32_t)npix, b->gs[i].spp);
        vdbc_status s = launch_check("batch pixel sums to image");
        if (s) return s;
    }
    return VDBC_OK;
}

static vdbc_status batch_enqueue(vdbc_batch* b, hipStream_t st)
{
    vdbc_status s;
    // the persistent launch builds every volume's majorant grid and coarse
    // bits in one launch each (below the grid-size limit); one launch per
    // volume otherwise, and for the per-volume baseline
    const bool batched_pre = b->t.persistent && b->cells_total < (1ull << 24) && b->cblocks_total < (1ull << 24);
    if (batched_pre) {
        hipLaunchKernelGGL(majorant_batch_kernel, dim3((unsigned)b->cells_total), dim3(kBlock), 0, st, b->d_descs,
                           b->d_cell_base, b->n);
        if ((s = launch_check("batched majorants"))) return s;
        hipLaunchKernelGGL(coarse_bits_batch_kernel, dim3((unsigned)b->cblocks_total), dim3(kBlock), 0, st,
                           b->d_descs, b->d_coarse_base, b->n);
        if ((s = launch_check("batched coarse occupancy"))) return s;
    }
    for (uint32_t i = 0; i < b->n; ++i) {
        if (!batched_pre) {
            if ((s = launch_majorant<VdbAcc>(b->views[i], b->meds[i], (uint32_t)b->gs[i].C, b->majs[i], st)))
                return s;
            const PtArgs& g = b->gs[i];
            const uint64_t ncoarse = (uint64_t)g.cgx * g.cgy * g.cgz;
            hipLaunchKernelGGL(coarse_bits_kernel, dim3((unsigned)((ncoarse + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                               st, b->majs[i], g, b->coarse[i]);
            if ((s = launch_check("batch coarse occupancy"))) return s;
        }
        if (b->sums[i].rgbn) {
            const uint64_t words = batch_sums_bytes((uint64_t)b->cams[i].width * b->cams[i].height) / 16;
            hipLaunchKernelGGL(pt_sums_clear_kernel,
                               dim3((unsigned)std::min<uint64_t>((words + kBlock - 1) / kBlock, 4096)), dim3(kBlock), 0,
                               st, reinterpret_cast<uint4*>(b->sums[i].rgbn), words);
            if ((s = launch_check("batch pixel sums clear"))) return s;
        }
    }
    if (b->t.persistent) {
        hipLaunchKernelGGL(zero_u32, dim3(1), dim3(64), 0, st, b->d_counter);
        hipLaunchKernelGGL(pt_batch_kernel, dim3(b->grid_blocks), dim3(kBlock), 4u * (size_t)b->max_cwords, st,
                           b->d_descs, b->d_items, b->n_items, b->d_counter);
        if ((s = launch_check("batched render"))) return s;
        return batch_resolve(b, st);
    }
    // one launch per volume; the launches run in stream order, so they share
    // the tile queue, cleared before each
    for (uint32_t i = 0; i < b->n; ++i) {
        const PtArgs& g = b->gs[i];
        const uint32_t items = (uint32_t)(b->tiles_x[i] * b->tiles_y[i]) * g.chunks;
        hipLaunchKernelGGL(zero_u32, dim3(1), dim3(64), 0, st, b->d_counter);
        const dim3 grid(std::min<uint32_t>(items, (uint32_t)b->grid_blocks));
        if (b->meds[i].env)
            hipLaunchKernelGGL((pt_kernel<VdbAcc, VdbView, false, false, true>), grid, dim3(kBlock),
                               4u * (size_t)g.cwords, st, b->views[i], b->cams[i], b->meds[i], g, b->majs[i],
                               b->coarse[i], b->images[i], nullptr, nullptr, b->d_counter, b->sums[i], nullptr);
        else
            hipLaunchKernelGGL((pt_kernel<VdbAcc, VdbView, false, false, false>), grid, dim3(kBlock),
                               4u * (size_t)g.cwords, st, b->views[i], b->cams[i], b->meds[i], g, b->majs[i],
                               b->coarse[i], b->images[i], nullptr, nullptr, b->d_counter, b->sums[i], nullptr);
        if ((s = launch_check("per-volume render"))) return s;
    }
    return batch_resolve(b, st);
}

}  // namespace vdbc

extern "C" vdbc_status vdbc_batch_workspace(const vdbc_batch_item* items, uint32_t n, const vdbc_tuning* t,
                                            uint64_t* bytes)
{
    clear_error();
    if (!bytes) return fail(VDBC_E_INVALID, "null argument");
    vdbc_tuning tt;
    vdbc_status s = batch_tuning(t, &tt);
    if (s) return s;
    vdbc_batch b;
    std::vector<uint64_t> mo, co, so;
    uint64_t io, total;
    if ((s = batch_plan(items, n, tt, &b, &mo, &co, &so, &io, &total))) return s;
    *bytes = total;
    return VDBC_OK;
}

extern "C" vdbc_status vdbc_batch_create(const vdbc_batch_item* items, uint32_t n, const vdbc_tuning* t, void* ws,
                                         uint64_t ws_bytes, void* stream, vdbc_batch** out)
{
    clear_error();
    if (!out || !ws) return fail(VDBC_E_INVALID, "null argument");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(VDBC_E_INVALID, "workspace must be 256-byte aligned");
    *out = nullptr;
    vdbc_tuning tt;
    vdbc_status s = batch_tuning(t, &tt);
    if (s) return s;
    std::unique_ptr<vdbc_batch> b(new (std::nothrow) vdbc_batch());
    if (!b) return fail(VDBC_E_NOMEM, "no memory");
    std::vector<uint64_t> mo, co, so;
    uint64_t io, total;
    if ((s = batch_plan(items, n, tt, b.get(), &mo, &co, &so, &io, &total))) return s;
    if (ws_bytes < total)
        return fail(VDBC_E_BUFFER_TOO_SMALL, "batch workspace needs %llu bytes", (unsigned long long)total);
    uint8_t* w = static_cast<uint8_t*>(ws);
    b->d_counter = reinterpret_cast<uint32_t*>(w);
    b->d_descs = reinterpret_cast<BatchDesc*>(w + 256);
    b->d_cell_base = reinterpret_cast<uint32_t*>(w + 256 + align256((uint64_t)n * sizeof(BatchDesc)));
    b->d_coarse_base = b->d_cell_base + (n + 1);
    b->d_items = reinterpret_cast<uint32_t*>(w + io);
    for (uint32_t i = 0; i < n; ++i) {
        b->majs.push_back(reinterpret_cast<float*>(w + mo[i]));
        b->coarse.push_back(reinterpret_cast<uint32_t*>(w + co[i]));
        b->sums.push_back(so[i] ? PtSums{reinterpret_cast<unsigned long long*>(w + so[i]), nullptr} : PtSums{});
    }
    // descriptors and the cost-ordered work list (largest estimated cost first:
    // samples per pixel x ray length through the volume)
    std::vector<BatchDesc> descs(n);
    std::vector<uint32_t> order(n);
    for (uint32_t i = 0; i < n; ++i) {
        descs[i] = BatchDesc{b->views[i], b->cams[i], b->meds[i], b->gs[i], b->majs[i], b->coarse[i], b->images[i],
                             b->sums[i], b->tiles_x[i]};
        order[i] = i;
    }
    auto cost = [&](uint32_t i) {
        return (double)b->gs[i].spp * (double)(b->views[i].nx + b->views[i].ny + b->views[i].nz);
    };
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t c) { return cost(a) > cost(c); });
    std::vector<uint32_t> list;
    list.reserve(b->n_items);
    for (uint32_t i : order)
        for (uint32_t k = 0; k < (uint32_t)(b->tiles_x[i] * b->tiles_y[i]) * b->gs[i].chunks; ++k)
            list.push_back((i << 20) | k);
    // prefix tables of the batched majorant launches: macrocells and
    // coarse-bit workgroups per volume (the launch is used only while both
    // totals stay below 2^24 workgroups)
    std::vector<uint32_t> bases(2 * (size_t)(n + 1), 0u);
    for (uint32_t i = 0; i < n; ++i) {
        const PtArgs& g = b->gs[i];
        b->cells_total += (uint64_t)g.gx * g.gy * g.gz;
        b->cblocks_total += ((uint64_t)g.cgx * g.cgy * g.cgz + kBlock - 1) / kBlock;
        bases[i + 1] = (uint32_t)std::min<uint64_t>(b->cells_total, 0xFFFFFFFFull);
        bases[n + 1 + i + 1] = (uint32_t)std::min<uint64_t>(b->cblocks_total, 0xFFFFFFFFull);
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(b->d_cell_base, bases.data(), bases.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(b->d_descs, descs.data(), n * sizeof(BatchDesc), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(b->d_items, list.data(), list.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(VDBC_E_DEVICE, "batch descriptor upload: %s", hipGetErrorString(hipGetLastError()));
    b->grid_blocks = device_cus() * (int)tt.blocks_per_cu;
    *out = b.release();
    return VDBC_OK;
}

extern "C" vdbc_status vdbc_batch_launch(vdbc_batch* b, void* stream)
{
    clear_error();
    if (!b) return fail(VDBC_E_INVALID, "null batch");
    return batch_enqueue(b, static_cast<hipStream_t>(stream));
}

extern "C" vdbc_status vdbc_batch_capture(vdbc_batch* b, void* stream)
{
    clear_error();
    if (!b) return fail(VDBC_E_INVALID, "null batch");
    if (!stream) return fail(VDBC_E_INVALID, "capture needs a non-default stream");
    if (b->exec) return VDBC_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(VDBC_E_DEVICE, "begin capture: %s", hipGetErrorString(hipGetLastError()));
    vdbc_status s = batch_enqueue(b, st);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (s) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess || !g) return fail(VDBC_E_DEVICE, "end capture: %s", hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(VDBC_E_DEVICE, "graph instantiate failed");
    }
    b->graph = g;
    b->exec = ex;
    return VDBC_OK;
}

extern "C" vdbc_status vdbc_batch_graph_launch(vdbc_batch* b, void* stream)
{
    clear_error();
    if (!b || !b->exec) return fail(VDBC_E_INVALID, "batch has no captured graph");
    if (hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)) != hipSuccess)
        return fail(VDBC_E_DEVICE, "graph launch: %s", hipGetErrorString(hipGetLastError()));
    return VDBC_OK;
}

extern "C" void vdbc_batch_destroy(vdbc_batch* b)
{
    if (!b) return;
    // teardown: nothing useful can be done with a failure here
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    delete b;
}
