/* Philox-4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11), bulk uniform
 * draws for the seeded input generator.
 *
 * One draw is a pure function of (seed, field, index, sub): the counter is
 * (index lo, index hi, sub, 0), the key (seed, field).  Each round maps the
 * counter (c0, c1, c2, c3) with the products M0 c0 = (hi0, lo0) and
 * M1 c2 = (hi1, lo1) to (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0), and the
 * key advances by the Weyl constants between rounds.  The first two words
 * give one 53-bit uniform in (0, 1), the last two a second one:
 * ((w0 >> 5) 2^26 + (w1 >> 6) + 1/2) / 2^53.  The values equal those of the
 * module's numpy implementation bit for bit (integer arithmetic and exact
 * double operations only).  Holds none of the solver's arithmetic. */
#include <stdint.h>

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

static void philox10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    for (int r = 0; r < 10; r++) {
        if (r) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        const uint64_t p0 = (uint64_t)PHILOX_M0 * c[0];
        const uint64_t p1 = (uint64_t)PHILOX_M1 * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

static double u53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6) + 0.5) / 9007199254740992.0;
}

/* raw words: out[4 i + q] = word q of index i (for the known-answer test) */
void philox_words(uint32_t seed, uint32_t field, const uint64_t *idx, int64_t n, uint32_t sub,
                  uint32_t *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        uint32_t c[4] = {(uint32_t)idx[i], (uint32_t)(idx[i] >> 32), sub, 0u};
        philox10(c, seed, field);
        for (int q = 0; q < 4; q++) out[4 * i + q] = c[q];
    }
}

/* u1[i], u2[i] = the two uniforms of index idx[i] (idx NULL: index
 * idx0 + i); u2 may be NULL */
void philox_uniforms(uint32_t seed, uint32_t field, const uint64_t *idx, uint64_t idx0, int64_t n,
                     uint32_t sub, double *u1, double *u2)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        const uint64_t id = idx ? idx[i] : idx0 + (uint64_t)i;
        uint32_t c[4] = {(uint32_t)id, (uint32_t)(id >> 32), sub, 0u};
        philox10(c, seed, field);
        u1[i] = u53(c[0], c[1]);
        if (u2) u2[i] = u53(c[2], c[3]);
    }
}
