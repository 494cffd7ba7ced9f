/* Philox4x32-10 counter-based generator, written from its published
 * definition: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
 * 1, 2, 3", SC'11, Section 4 (Philox S-box with multipliers 0xD2511F53 and
 * 0xCD9E8D57, Weyl key schedule 0x9E3779B9 / 0xBB67AE85, 10 rounds).
 * TEST INFRASTRUCTURE ONLY (see oracle.h). */
#include "oracle.h"

static void round4(uint32_t c[4], const uint32_t k[2])
{
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

void ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        round4(c, k);
    }
    out[0] = c[0];
    out[1] = c[1];
    out[2] = c[2];
    out[3] = c[3];
}

/* The generator applied to n (counter, key) pairs, one after another. */
void ref_philox_many(const uint32_t* ctr, const uint32_t* key, uint64_t n, uint32_t* out)
{
    for (uint64_t i = 0; i < n; ++i) ref_philox4x32_10(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

/* 24 high bits -> [0, 1) with spacing 2^-24. */
double ref_u01(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }
