/* Oracle field access: walking the canonical buffer from the root to a leaf
 * (the VDB random access of Section 2.3 / Section 3.2.2), nearest and
 * trilinear reconstruction at level 0 with the background value substituted
 * where no voxel exists (Section 3.2.2), and the same reconstruction on a plain
 * dense array (the "3D texture" of Section 5.3, read in software).
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Sample convention: positions are in index space with voxel centres on the
 * integers; a corner outside [0, dims) or without a voxel reads B.  Trilinear
 * = lerp along x, then y, then z with lerp(a,b,t) = a + t*(b-a), evaluated in
 * double from the float corner values. */
#include <math.h>
#include <string.h>

#include "oracle.h"

static uint32_t rd32(const uint8_t* p)
{
    uint32_t v;
    memcpy(&v, p, 4);
    return v;
}
static uint64_t rd64(const uint8_t* p)
{
    uint64_t v;
    memcpy(&v, p, 8);
    return v;
}
static float rdf(const uint8_t* p)
{
    float v;
    memcpy(&v, p, 4);
    return v;
}

int ref_field_vdb(ref_field* f, const uint8_t* buf, uint64_t bytes)
{
    if (!buf || bytes < 256 || memcmp(buf, "VDBC", 4) != 0 || rd32(buf + 4) != 1)
        return REF_E_FORMAT;
    if (rd64(buf + 152) > bytes) return REF_E_FORMAT;
    f->kind = 0;
    f->buf = buf;
    f->bytes = bytes;
    f->dense = 0;
    f->nx = rd32(buf + 8);
    f->ny = rd32(buf + 12);
    f->nz = rd32(buf + 16);
    f->background = rdf(buf + 20);
    return REF_OK;
}

void ref_field_dense(ref_field* f, const float* dense, uint32_t nx, uint32_t ny,
                     uint32_t nz, float background)
{
    f->kind = 1;
    f->buf = 0;
    f->bytes = 0;
    f->dense = dense;
    f->nx = nx;
    f->ny = ny;
    f->nz = nz;
    f->background = background;
}

static int popc64(uint64_t x)
{
    int c = 0;
    while (x) {
        x &= x - 1;
        ++c;
    }
    return c;
}

/* One internal-node level: slot n inside the node at `node` (array of 32-byte
 * word records).  Returns 1 = child (index in *idx), 2 = tile (index in *idx),
 * 0 = nothing there. */
static int node_slot(const uint8_t* node, uint32_t n, uint32_t* idx)
{
    const uint8_t* rec = node + (uint64_t)(n / 64) * 32u;
    uint64_t below = ((uint64_t)1 << (n % 64)) - 1u;
    uint64_t child = rd64(rec), tile = rd64(rec + 16);
    if ((child >> (n % 64)) & 1u) {
        *idx = rd32(rec + 8) + (uint32_t)popc64(child & below);
        return 1;
    }
    if ((tile >> (n % 64)) & 1u) {
        *idx = rd32(rec + 12) + (uint32_t)popc64(tile & below);
        return 2;
    }
    return 0;
}

float ref_lookup(const ref_field* f, int64_t i, int64_t j, int64_t k)
{
    if (i < 0 || j < 0 || k < 0 || i >= f->nx || j >= f->ny || k >= f->nz)
        return f->background;
    if (f->kind == 1) return f->dense[i + (int64_t)f->nx * (j + (int64_t)f->ny * k)];
    const uint8_t* b = f->buf;
    uint32_t rnx = rd32(b + 84), rny = rd32(b + 88);
    uint64_t root = rd64(b + 96);
    uint32_t u = rd32(b + root + 4 * ((i >> 12) + rnx * ((j >> 12) + (uint64_t)rny * (k >> 12))));
    if (u == 0xFFFFFFFFu) return f->background;
    const uint8_t* unode = b + rd64(b + 104) + (uint64_t)u * 512u * 32u;
    uint32_t n1 = (uint32_t)(((i >> 7) & 31) + 32 * (((j >> 7) & 31) + 32 * ((k >> 7) & 31)));
    uint32_t idx;
    int s = node_slot(unode, n1, &idx);
    if (s == 0) return f->background;
    if (s == 2) return rdf(b + rd64(b + 120) + 4u * (uint64_t)idx);
    const uint8_t* lnode = b + rd64(b + 112) + (uint64_t)idx * 64u * 32u;
    uint32_t n2 = (uint32_t)(((i >> 3) & 15) + 16 * (((j >> 3) & 15) + 16 * ((k >> 3) & 15)));
    s = node_slot(lnode, n2, &idx);
    if (s == 0) return f->background;
    if (s == 2) return rdf(b + rd64(b + 128) + 4u * (uint64_t)idx);
    uint32_t n3 = (uint32_t)((i & 7) + 8 * ((j & 7) + 8 * (k & 7)));
    return rdf(b + rd64(b + 144) + 2048u * (uint64_t)idx + 4u * n3);
}

void ref_lookup_many(const ref_field* f, const int64_t* ijk, uint64_t n, float* out)
{
    for (uint64_t q = 0; q < n; ++q)
        out[q] = ref_lookup(f, ijk[3 * q], ijk[3 * q + 1], ijk[3 * q + 2]);
}

static double lerp(double a, double b, double t) { return a + t * (b - a); }

double ref_sample(const ref_field* f, const float p[3], uint32_t filter)
{
    double fl[3], fr[3];
    int64_t i0[3];
    for (int a = 0; a < 3; ++a) {
        fl[a] = floor((double)p[a]);
        i0[a] = (int64_t)fl[a];
        fr[a] = (double)p[a] - fl[a];
    }
    if (filter == 0) { /* nearest voxel centre, halves rounded up */
        return (double)ref_lookup(f, i0[0] + (fr[0] >= 0.5), i0[1] + (fr[1] >= 0.5),
                                  i0[2] + (fr[2] >= 0.5));
    }
    double c[2][2][2];
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx)
                c[dz][dy][dx] = (double)ref_lookup(f, i0[0] + dx, i0[1] + dy, i0[2] + dz);
    double y0 = lerp(lerp(c[0][0][0], c[0][0][1], fr[0]), lerp(c[0][1][0], c[0][1][1], fr[0]), fr[1]);
    double y1 = lerp(lerp(c[1][0][0], c[1][0][1], fr[0]), lerp(c[1][1][0], c[1][1][1], fr[0]), fr[1]);
    return lerp(y0, y1, fr[2]);
}

void ref_sample_many(const ref_field* f, const float* pos, uint64_t n, uint32_t filter,
                     double* out)
{
    for (uint64_t q = 0; q < n; ++q) out[q] = ref_sample(f, pos + 3 * q, filter);
}
