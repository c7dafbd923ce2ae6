/*
 * philox.c -- Philox4x32-10 counter-based generator for the oracle.
 *
 * TEST INFRASTRUCTURE ONLY (see u1_oracle.h).
 *
 * Written from the description in J. K. Salmon, M. A. Moraes, R. O. Dror,
 * D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11, Sec. 4.2:
 * each round multiplies counter words 0 and 2 by two fixed 32-bit odd
 * constants, takes the 64-bit products apart into high and low halves, xors
 * the high halves with the other two counter words and the round key, and
 * permutes the four words; the two key words are bumped by the Weyl constants
 * (golden ratio and sqrt(3) - 1, in 32-bit fixed point) between rounds.
 * Ten rounds are used.  The paper itself draws its numbers from CURAND
 * (Sec. II.D); a counter-based stream replaces that stateful generator.
 */
#include "u1_oracle.h"

static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u;
static const uint32_t PHILOX_W1 = 0xBB67AE85u;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}
