/* Oracle renderers (Section 4): majorant macrocell grid, emission-absorption
 * ray marching, and a delta-tracking (Woodcock) volumetric path tracer that
 * walks the majorant grid with a 3D-DDA and tracks free-flight distances
 * inside non-empty cells.  Double precision throughout.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Scene conventions (readings; the paper fixes none of them):
 *  - the volume occupies the index-space box [-0.5, n-0.5]^3;
 *  - extinction sigma(s) = sigma_scale / max(nx,ny,nz) * alpha_TF(s) per voxel
 *    length, where alpha_TF is the alpha channel of a piecewise-linear RGBA
 *    transfer function (Section 4: alpha serves as extinction);
 *  - macrocells are C^3 voxels, cell c covering [C*c-0.5, C*(c+1)-0.5); the
 *    majorant of a cell is the maximum of sigma over the value range of the
 *    voxels [C*c-1, C*c+C] (one-voxel dilation covers every trilinear
 *    footprint whose sample lies in the cell);
 *  - path tracer: albedo times TF colour as throughput weight at each real
 *    collision, next-event estimation towards one directional light with a
 *    binary delta-tracked shadow transmittance, isotropic phase 1/(4 pi),
 *    fixed bounce cap, constant ambient radiance added on escape;
 *  - random numbers: Philox4x32-10 with key (seed_lo ^ pixel, seed_hi) and
 *    counter (block, sample, stream << 16 | bounce, frame); draw d of a
 *    (sample, bounce, stream) is word d & 3 of block d >> 2.  Stream 0 of
 *    bounce b is path segment b: its first two draws choose the segment's
 *    direction (the pixel jitter for b = 0, the isotropic scattering
 *    direction after collision b - 1 otherwise), the rest are its free
 *    flights.  Stream 1 of bounce b is the shadow ray cast from collision b.
 *  - image-based light (optional, reading R25): an escaping path sees the
 *    radiance of a lat-long map, nearest texel at u = (atan2(d_z, d_x) + pi) /
 *    (2 pi), v = acos(d_y) / pi, instead of the constant ambient;
 *  - Russian roulette (optional, reading R24): a segment b >= 1 then opens
 *    with one more draw u; from b = 2 on the path survives with probability
 *    q = min(1, max(beta)) (u < q) and its throughput is divided by q; the
 *    direction takes the next two draws.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define PI_D 3.14159265358979323846

/* ------------------------------ helpers ------------------------------ */

typedef struct {
    uint32_t key[2];
    uint32_t sample, bounce, stream, frame;
    uint32_t d;
    uint32_t cache[4];
    uint32_t block;
    int have;
} rng_t;

static void rng_init(rng_t* r, uint64_t seed, uint32_t pixel, uint32_t sample,
                     uint32_t bounce, uint32_t stream, uint32_t frame)
{
    r->key[0] = (uint32_t)seed ^ pixel;
    r->key[1] = (uint32_t)(seed >> 32);
    r->sample = sample;
    r->bounce = bounce;
    r->stream = stream;
    r->frame = frame;
    r->d = 0;
    r->have = 0;
}

static double rng_next(rng_t* r)
{
    uint32_t block = r->d >> 2;
    if (!r->have || r->block != block) {
        uint32_t ctr[4] = {block, r->sample, (r->stream << 16) | r->bounce, r->frame};
        ref_philox4x32_10(ctr, r->key, r->cache);
        r->block = block;
        r->have = 1;
    }
    uint32_t w = r->cache[r->d & 3];
    r->d++;
    return ref_u01(w);
}

static void tf_eval(const ref_medium* m, double s, double out[4])
{
    double x = (s - (double)m->tf_lo) / ((double)m->tf_hi - (double)m->tf_lo);
    if (x < 0.0) x = 0.0;
    if (x > 1.0) x = 1.0;
    double pos = x * (double)(m->tf_n - 1);
    int i = (int)floor(pos);
    if (i > (int)m->tf_n - 2) i = (int)m->tf_n - 2;
    double fr = pos - (double)i;
    for (int c = 0; c < 4; ++c)
        out[c] = (double)m->tf[i][c] + fr * ((double)m->tf[i + 1][c] - (double)m->tf[i][c]);
}

static double density_scale(const ref_field* f, const ref_medium* m)
{
    uint32_t nmax = f->nx;
    if (f->ny > nmax) nmax = f->ny;
    if (f->nz > nmax) nmax = f->nz;
    return (double)m->sigma_scale / (double)nmax;
}

static double sigma_of(const ref_field* f, const ref_medium* m, double s)
{
    double c[4];
    tf_eval(m, s, c);
    return density_scale(f, m) * c[3];
}

/* trilinear sample at a double-precision position (same rule as ref_sample) */
static double sample_d(const ref_field* f, const double p[3])
{
    double fl[3], fr[3];
    int64_t i0[3];
    for (int a = 0; a < 3; ++a) {
        fl[a] = floor(p[a]);
        i0[a] = (int64_t)fl[a];
        fr[a] = p[a] - fl[a];
    }
    double c[2][2][2];
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx)
                c[dz][dy][dx] = (double)ref_lookup(f, i0[0] + dx, i0[1] + dy, i0[2] + dz);
#define LERP(a, b, t) ((a) + (t) * ((b) - (a)))
    double y0 = LERP(LERP(c[0][0][0], c[0][0][1], fr[0]), LERP(c[0][1][0], c[0][1][1], fr[0]), fr[1]);
    double y1 = LERP(LERP(c[1][0][0], c[1][0][1], fr[0]), LERP(c[1][1][0], c[1][1][1], fr[0]), fr[1]);
    return LERP(y0, y1, fr[2]);
#undef LERP
}

/* ray / box [-0.5, n-0.5]^3; returns 1 and [t0,t1] (t0 >= 0) if non-empty */
static int box_clip(const ref_field* f, const double o[3], const double d[3], double* t0,
                    double* t1)
{
    double n[3] = {(double)f->nx, (double)f->ny, (double)f->nz};
    double lo = -INFINITY, hi = INFINITY;
    for (int a = 0; a < 3; ++a) {
        double bl = -0.5, bh = n[a] - 0.5;
        if (d[a] == 0.0) {
            if (o[a] < bl || o[a] > bh) return 0;
            continue;
        }
        double ta = (bl - o[a]) / d[a], tb = (bh - o[a]) / d[a];
        double tn = ta < tb ? ta : tb, tf = ta < tb ? tb : ta;
        if (tn > lo) lo = tn;
        if (tf < hi) hi = tf;
    }
    if (lo < 0.0) lo = 0.0;
    *t0 = lo;
    *t1 = hi;
    return lo < hi;
}

/* ------------------------------ majorant ------------------------------ */

static double alpha_max(const ref_medium* m, double a, double b)
{
    double c[4];
    tf_eval(m, a, c);
    double best = c[3];
    tf_eval(m, b, c);
    if (c[3] > best) best = c[3];
    for (uint32_t i = 0; i < m->tf_n; ++i) {
        double s = (double)m->tf_lo +
                   (double)i * ((double)m->tf_hi - (double)m->tf_lo) / (double)(m->tf_n - 1);
        if (s > a && s < b && (double)m->tf[i][3] > best) best = (double)m->tf[i][3];
    }
    return best;
}

int ref_majorant_cells(const ref_field* f, const ref_medium* m, uint32_t C, uint64_t begin,
                       uint64_t end, double* maj)
{
    if (C == 0 || m->tf_n < 2 || m->tf_n > 64) return REF_E_INVALID;
    uint64_t gx = (f->nx + C - 1) / C, gy = (f->ny + C - 1) / C, gz = (f->nz + C - 1) / C;
    if (begin > end || end > gx * gy * gz) return REF_E_INVALID;
    double ds = density_scale(f, m);
    for (uint64_t cell = begin; cell < end; ++cell) {
        int64_t cx = (int64_t)(cell % gx), cy = (int64_t)((cell / gx) % gy), cz = (int64_t)(cell / (gx * gy));
        double vmin = INFINITY, vmax = -INFINITY;
        for (int64_t k = (int64_t)C * cz - 1; k <= (int64_t)C * cz + C; ++k)
            for (int64_t j = (int64_t)C * cy - 1; j <= (int64_t)C * cy + C; ++j)
                for (int64_t i = (int64_t)C * cx - 1; i <= (int64_t)C * cx + C; ++i) {
                    double v = (double)ref_lookup(f, i, j, k);
                    if (v < vmin) vmin = v;
                    if (v > vmax) vmax = v;
                }
        maj[cell] = ds * alpha_max(m, vmin, vmax);
    }
    return REF_OK;
}

int ref_majorant(const ref_field* f, const ref_medium* m, uint32_t C, double* maj)
{
    if (C == 0) return REF_E_INVALID;
    uint64_t cells = (uint64_t)((f->nx + C - 1) / C) * ((f->ny + C - 1) / C) * ((f->nz + C - 1) / C);
    return ref_majorant_cells(f, m, C, 0, cells, maj);
}

/* --------------------------- emission-absorption --------------------------- */

static void camera_ray(const ref_camera* c, double px, double py, double o[3], double d[3])
{
    double len = 0.0;
    for (int a = 0; a < 3; ++a) {
        if (c->kind == 1) {
            o[a] = (double)c->origin[a];
            d[a] = (double)c->lower_left[a] + px * (double)c->du[a] + py * (double)c->dv[a];
        } else {
            o[a] = (double)c->lower_left[a] + px * (double)c->du[a] + py * (double)c->dv[a];
            d[a] = (double)c->dir[a];
        }
        len += d[a] * d[a];
    }
    len = sqrt(len);
    for (int a = 0; a < 3; ++a) d[a] /= len;
}

int ref_render_ea(const ref_field* f, const ref_camera* c, const ref_medium* m,
                  const ref_render_params* r, double* image)
{
    if (!(r->step > 0.0f) || m->tf_n < 2 || m->tf_n > 64) return REF_E_INVALID;
    double ds = density_scale(f, m);
    double step = (double)r->step;
    for (uint32_t py = 0; py < c->height; ++py)
        for (uint32_t px = 0; px < c->width; ++px) {
            double o[3], d[3], t0, t1;
            camera_ray(c, px + 0.5, py + 0.5, o, d);
            double col[3] = {0, 0, 0}, T = 1.0;
            if (box_clip(f, o, d, &t0, &t1)) {
                for (uint64_t k = 0;; ++k) {
                    double t = t0 + ((double)k + 0.5) * step;
                    if (t >= t1) break;
                    double x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
                    double s = sample_d(f, x);
                    double tf[4];
                    tf_eval(m, s, tf);
                    double a = 1.0 - exp(-ds * tf[3] * step);
                    for (int ch = 0; ch < 3; ++ch) col[ch] += T * a * tf[ch];
                    T *= 1.0 - a;
                    if (T < (double)r->t_terminate) break;
                }
            }
            double* out = image + 4 * ((uint64_t)py * c->width + px);
            out[0] = col[0];
            out[1] = col[1];
            out[2] = col[2];
            out[3] = 1.0 - T;
        }
    return REF_OK;
}

/* Implicit iso-surface marcher (reading R22): plain lattice march, sign
 * test between consecutive samples, bisection, central-difference normal. */
int ref_render_iso(const ref_field* f, const ref_camera* c, double iso, double step,
                   uint32_t refine, double* image, double* aux)
{
    if (!(step > 0.0) || refine > 64) return REF_E_INVALID;
    for (uint32_t py = 0; py < c->height; ++py)
        for (uint32_t px = 0; px < c->width; ++px) {
            double o[3], d[3], t0, t1;
            camera_ray(c, px + 0.5, py + 0.5, o, d);
            double* out = image + 4 * ((uint64_t)py * c->width + px);
            out[0] = out[1] = out[2] = out[3] = 0.0;
            double m_lat = INFINITY, m_mid = INFINITY, thit = -1.0;
            if (box_clip(f, o, d, &t0, &t1)) {
                int have = 0, prev = 0;
                double tprev = 0.0;
                for (uint64_t k = 0;; ++k) {
                    double t = t0 + ((double)k + 0.5) * step;
                    if (t >= t1) break;
                    double x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
                    double v = sample_d(f, x);
                    if (fabs(v - iso) < m_lat) m_lat = fabs(v - iso);
                    int inside = v >= iso;
                    if (have && inside != prev) {
                        double lo = tprev, hi = t;
                        for (uint32_t it = 0; it < refine; ++it) {
                            double mid = 0.5 * (lo + hi);
                            double y[3] = {o[0] + mid * d[0], o[1] + mid * d[1], o[2] + mid * d[2]};
                            double w = sample_d(f, y);
                            if (fabs(w - iso) < m_mid) m_mid = fabs(w - iso);
                            if ((w >= iso) == prev) lo = mid;
                            else hi = mid;
                        }
                        double th = 0.5 * (lo + hi);
                        thit = th;
                        double p[3] = {o[0] + th * d[0], o[1] + th * d[1], o[2] + th * d[2]};
                        double g[3];
                        for (int a = 0; a < 3; ++a) {
                            double pp[3] = {p[0], p[1], p[2]}, pm[3] = {p[0], p[1], p[2]};
                            pp[a] += 0.5;
                            pm[a] -= 0.5;
                            g[a] = sample_d(f, pp) - sample_d(f, pm);
                        }
                        double len = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
                        for (int a = 0; a < 3; ++a) out[a] = len > 0.0 ? 0.5 * (1.0 - g[a] / len) : 0.5;
                        out[3] = 1.0;
                        break;
                    }
                    have = 1;
                    prev = inside;
                    tprev = t;
                }
            }
            if (aux) {
                double* x = aux + 3 * ((uint64_t)py * c->width + px);
                x[0] = thit;
                x[1] = m_lat;
                x[2] = m_mid;
            }
        }
    return REF_OK;
}

/* Isotropic phase function sampling: uniform direction on the unit sphere
 * from two uniforms (z = 1 - 2u, phi = 2 pi u'). */
void ref_isotropic(double u1, double u2, double d[3])
{
    double z = 1.0 - 2.0 * u1;
    double phi = 2.0 * PI_D * u2;
    double rr = sqrt(z * z < 1.0 ? 1.0 - z * z : 0.0);
    d[0] = rr * cos(phi);
    d[1] = rr * sin(phi);
    d[2] = z;
}

/* ------------------------------ delta tracking ------------------------------ */

typedef struct {
    const ref_field* f;
    const ref_medium* m;
    const double* maj;
    uint32_t C;
    int64_t g[3];
} tracker;

/* Free-flight distance by delta tracking over the majorant grid, walked with
 * a 3D-DDA; returns 1 with the collision distance, 0 if the ray leaves. */
static int free_flight(const tracker* tk, const double o[3], const double d[3], double t0,
                       double t1, rng_t* rng, double* t_hit)
{
    if (!(t0 < t1)) return 0;
    int64_t cell[3], step[3];
    double C = (double)tk->C;
    for (int a = 0; a < 3; ++a) {
        double p = o[a] + t0 * d[a];
        int64_t c = (int64_t)floor((p + 0.5) / C);
        if (c < 0) c = 0;
        if (c > tk->g[a] - 1) c = tk->g[a] - 1;
        cell[a] = c;
        step[a] = d[a] > 0.0 ? 1 : (d[a] < 0.0 ? -1 : 0);
    }
    double t = t0;
    for (;;) {
        double te = t1;
        int axis = -1;
        for (int a = 0; a < 3; ++a) {
            if (d[a] == 0.0) continue;
            double bnd = C * (double)(cell[a] + (d[a] > 0.0 ? 1 : 0)) - 0.5;
            double ta = (bnd - o[a]) / d[a];
            if (ta < te) {
                te = ta;
                axis = a;
            }
        }
        double mu = tk->maj[cell[0] + tk->g[0] * (cell[1] + tk->g[1] * cell[2])];
        if (mu > 0.0 && t < te) {
            for (;;) {
                t = t - log(1.0 - rng_next(rng)) / mu;
                if (t >= te) break;
                double x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
                double sig = sigma_of(tk->f, tk->m, sample_d(tk->f, x));
                if (rng_next(rng) * mu < sig) {
                    *t_hit = t;
                    return 1;
                }
            }
        }
        if (axis < 0) return 0;
        t = te;
        cell[axis] += step[axis];
        if (cell[axis] < 0 || cell[axis] >= tk->g[axis]) return 0;
    }
}

static void tracker_grid(tracker* tk, const ref_field* f, const ref_medium* m, uint32_t C)
{
    tk->f = f;
    tk->m = m;
    tk->C = C;
    tk->g[0] = (f->nx + C - 1) / C;
    tk->g[1] = (f->ny + C - 1) / C;
    tk->g[2] = (f->nz + C - 1) / C;
}

static int make_tracker(tracker* tk, const ref_field* f, const ref_medium* m, uint32_t C,
                        double** maj_out)
{
    if (C == 0) return REF_E_INVALID;
    tracker_grid(tk, f, m, C);
    double* maj = (double*)malloc(sizeof(double) * tk->g[0] * tk->g[1] * tk->g[2]);
    if (!maj) return REF_E_NOMEM;
    int rc = ref_majorant(f, m, C, maj);
    if (rc) {
        free(maj);
        return rc;
    }
    tk->maj = maj;
    *maj_out = maj;
    return REF_OK;
}

double ref_transmittance(const ref_field* f, const ref_medium* m, uint32_t C,
                         const float o[3], const float d[3], uint64_t trials, uint64_t seed)
{
    tracker tk;
    double* maj = NULL;
    if (make_tracker(&tk, f, m, C, &maj)) return NAN;
    double od[3] = {o[0], o[1], o[2]}, dd[3] = {d[0], d[1], d[2]};
    double t0, t1;
    double sum = 0.0;
    if (box_clip(f, od, dd, &t0, &t1)) {
        for (uint64_t i = 0; i < trials; ++i) {
            rng_t rng;
            rng_init(&rng, seed, (uint32_t)i, (uint32_t)(i >> 32), 0, 0, 0);
            double th;
            sum += free_flight(&tk, od, dd, t0, t1, &rng, &th) ? 0.0 : 1.0;
        }
    } else {
        sum = (double)trials;
    }
    free(maj);
    return sum / (double)trials;
}

/* Radiance seen by a ray leaving the volume along unit direction d: the
 * constant ambient, or the nearest texel of the lat-long map (R25). */
static void escape_radiance(const ref_medium* m, const double d[3], double out[3])
{
    if (!m->env) {
        for (int ch = 0; ch < 3; ++ch) out[ch] = (double)m->ambient[ch];
        return;
    }
    double u = (atan2(d[2], d[0]) + PI_D) / (2.0 * PI_D);
    double y = d[1] < -1.0 ? -1.0 : d[1] > 1.0 ? 1.0 : d[1];
    double v = acos(y) / PI_D;
    int64_t tx = (int64_t)floor(u * (double)m->env_w), ty = (int64_t)floor(v * (double)m->env_h);
    if (tx > (int64_t)m->env_w - 1) tx = (int64_t)m->env_w - 1;
    if (ty > (int64_t)m->env_h - 1) ty = (int64_t)m->env_h - 1;
    if (tx < 0) tx = 0;
    if (ty < 0) ty = 0;
    const float* p = m->env + 3 * ((uint64_t)ty * m->env_w + (uint64_t)tx);
    for (int ch = 0; ch < 3; ++ch) out[ch] = (double)p[ch];
}

static int render_pt(const tracker* tkp, const ref_camera* c, const ref_medium* m,
                     const ref_render_params* r, const uint32_t* pixels, uint64_t n_pixels,
                     double* rgba, double* aov);

int ref_render_pt(const ref_field* f, const ref_camera* c, const ref_medium* m,
                  const ref_render_params* r, const uint32_t* pixels, uint64_t n_pixels,
                  double* rgba, double* aov)
{
    if (r->spp == 0 || r->max_bounces == 0 || m->tf_n < 2 || m->tf_n > 64) return REF_E_INVALID;
    tracker tk;
    double* maj = NULL;
    int rc = make_tracker(&tk, f, m, r->macrocell, &maj);
    if (rc) return rc;
    rc = render_pt(&tk, c, m, r, pixels, n_pixels, rgba, aov);
    free(maj);
    return rc;
}

int ref_render_pt_majorant(const ref_field* f, const ref_camera* c, const ref_medium* m,
                           const ref_render_params* r, const double* maj, const uint32_t* pixels,
                           uint64_t n_pixels, double* rgba, double* aov)
{
    if (r->spp == 0 || r->max_bounces == 0 || m->tf_n < 2 || m->tf_n > 64 || r->macrocell == 0 || !maj)
        return REF_E_INVALID;
    tracker tk;
    tracker_grid(&tk, f, m, r->macrocell);
    tk.maj = maj;
    return render_pt(&tk, c, m, r, pixels, n_pixels, rgba, aov);
}

static int render_pt(const tracker* tkp, const ref_camera* c, const ref_medium* m,
                     const ref_render_params* r, const uint32_t* pixels, uint64_t n_pixels,
                     double* rgba, double* aov)
{
    const tracker tk = *tkp;
    const ref_field* f = tk.f;
    const double inv4pi = 1.0 / (4.0 * PI_D);
    double ld[3] = {m->light_dir[0], m->light_dir[1], m->light_dir[2]};
    for (uint64_t q = 0; q < n_pixels; ++q) {
        uint32_t pix = pixels[q];
        uint32_t px = pix % c->width, py = pix / c->width;
        double acc[3] = {0, 0, 0}, opac = 0.0, depth = 0.0, trans = 0.0;
        for (uint32_t s = 0; s < r->spp; ++s) {
            double o[3], d[3];
            double L[3] = {0, 0, 0}, beta[3] = {1, 1, 1};
            for (uint32_t b = 0; b < r->max_bounces; ++b) {
                /* segment b: its direction, then its free flight */
                rng_t path;
                rng_init(&path, r->seed, pix, s, b, 0, r->frame);
                if (r->rr && b > 0) {
                    double u = rng_next(&path);
                    double q = 1.0;
                    if (b >= 2) {
                        q = beta[0] > beta[1] ? beta[0] : beta[1];
                        q = beta[2] > q ? beta[2] : q;
                        q = q < 1.0 ? q : 1.0;
                    }
                    if (!(u < q)) break;
                    for (int ch = 0; ch < 3; ++ch) beta[ch] /= q;
                }
                double u1 = rng_next(&path), u2 = rng_next(&path);
                if (b == 0)
                    camera_ray(c, (double)px + u1, (double)py + u2, o, d);
                else
                    ref_isotropic(u1, u2, d);   /* o = previous collision */
                double t0, t1, th = 0.0;
                int hit = box_clip(f, o, d, &t0, &t1) &&
                          free_flight(&tk, o, d, t0, t1, &path, &th);
                if (b == 0) {
                    if (hit) {
                        opac += 1.0;
                        depth += (th - t0) / (t1 - t0);
                    } else {
                        trans += 1.0;
                        depth += 1.0;
                    }
                }
                if (!hit) {
                    double env[3];
                    escape_radiance(m, d, env);
                    for (int ch = 0; ch < 3; ++ch) L[ch] += beta[ch] * env[ch];
                    break;
                }
                double x[3] = {o[0] + th * d[0], o[1] + th * d[1], o[2] + th * d[2]};
                double tf[4];
                tf_eval(m, sample_d(f, x), tf);
                for (int ch = 0; ch < 3; ++ch) beta[ch] *= (double)m->albedo * tf[ch];
                rng_t sh;
                rng_init(&sh, r->seed, pix, s, b, 1, r->frame);
                double s0, s1, sth;
                int blocked = box_clip(f, x, ld, &s0, &s1) &&
                              free_flight(&tk, x, ld, s0, s1, &sh, &sth);
                if (!blocked)
                    for (int ch = 0; ch < 3; ++ch)
                        L[ch] += beta[ch] * inv4pi * (double)m->light_E[ch];
                if (b + 1 == r->max_bounces) break;
                o[0] = x[0];
                o[1] = x[1];
                o[2] = x[2];
            }
            for (int ch = 0; ch < 3; ++ch) acc[ch] += L[ch];
        }
        double inv = 1.0 / (double)r->spp;
        rgba[4 * q + 0] = acc[0] * inv;
        rgba[4 * q + 1] = acc[1] * inv;
        rgba[4 * q + 2] = acc[2] * inv;
        rgba[4 * q + 3] = opac * inv;
        if (aov) {
            aov[2 * q + 0] = depth * inv;
            aov[2 * q + 1] = trans * inv;
        }
    }
    return REF_OK;
}
