/*
 * philox.c -- Philox4x32-10 counter-based generator, written from its published
 * definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
 * 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications with the
 * constants 0xD2511F53 and 0xCD9E8D57, key bumped by the Weyl increments
 * 0x9E3779B9 and 0xBB67AE85 between rounds.
 *
 * TEST INFRASTRUCTURE (oracle).  Pinned by the generator's published
 * known-answer vectors (tests/golden/philox4x32_10_kat.txt).
 *
 * The paper does not say which generator it uses; draws are counter addressed
 * so that the oracle and the GPU library see the same numbers without sharing
 * code.  A uniform is formed from two 32-bit words as ((hi<<21)|(lo>>11) + 0.5)
 * * 2^-53, which lies strictly inside (0,1).
 */
#include "ns_oracle.h"

static void philox_round(uint32_t c[4], const uint32_t k[2]) {
  uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
  uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
  uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  uint32_t n0 = hi1 ^ c[1] ^ k[0];
  uint32_t n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k[0] += 0x9E3779B9u;
      k[1] += 0xBB67AE85u;
    }
    philox_round(c, k);
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

static double u01_from_words(uint32_t hi, uint32_t lo) {
  uint64_t v = ((uint64_t)hi << 21) | (uint64_t)(lo >> 11);   /* 53 bits */
  return ((double)v + 0.5) * (1.0 / 9007199254740992.0);      /* 2^-53 */
}

void orc_uniform2(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, double out[2]) {
  uint32_t ctr[4] = {c0, c1, c2, c3};
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  out[0] = u01_from_words(w[0], w[1]);
  out[1] = u01_from_words(w[2], w[3]);
}
